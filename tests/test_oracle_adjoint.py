"""Pin of the oracle's adjoint-state gradient against central finite differences."""
import numpy as np

from oracle import adjoint
from paper_2308_13476_amd import workloads as W


def test_adjoint_gradient_matches_finite_differences():
    n = 16
    h = 1.0 / n
    c = W.grf_velocity(n, 5)
    k2_true = W.k2_from_velocity(c, 0.5)
    k2 = W.smooth_k2(k2_true, 0.1)
    srcs = W.top_row_sources(n, 2)
    f = W.point_source_rhs(n, srcs)
    row = W.receiver_row(n)
    d = adjoint.forward(k2_true, h, f)[:, row, :]
    g, _ = adjoint.gradient(k2, h, f, row, d)
    rng = np.random.default_rng(11)
    nodes = [(0, 5), (n, n), (3, 0)] + [tuple(rng.integers(1, n, size=2)) for _ in range(5)]
    scale = np.abs(g).max()
    for j, i in nodes:
        fd = adjoint.finite_difference(k2, h, f, row, d, (j, i))
        assert abs(fd - g[j, i]) <= 1e-5 * max(abs(fd), 1e-3 * scale), ((j, i), fd, g[j, i])
