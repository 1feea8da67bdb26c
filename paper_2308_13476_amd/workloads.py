"""Seeded synthetic inputs for the 2D Helmholtz multigrid solver.

This module builds problem *data* only: wavenumber fields k(x,y)^2 on the
vertex grid, point-source right-hand sides, source and receiver positions and
random test vectors. It contains none of the solver's arithmetic, so both the
GPU path and the CPU oracle draw their inputs from it.

Grid convention: n mesh intervals per side, h = 1/n, nodes (i, j) with
0 <= i, j <= n at x = i h, y = j h (y = 1 is the top). Fields are numpy arrays
of shape (n+1, n+1) indexed [j, i], so flattening in C order puts x fastest.

The model problems follow §2 of the paper (MP 2-A: constant k, a unit point
source at the centre; MP 2-B: k(x,y) varying between two bounds). The wedge
and Gaussian-random-field velocity models stand in for the paper's
unspecified variable-k profiles (its figures are not reproducible).
"""
from __future__ import annotations

import numpy as np


def grid_h(n: int) -> float:
    """Mesh width h = 1/n of the unit square with n intervals per side."""
    return 1.0 / n


def constant_k2(n: int, k: float) -> np.ndarray:
    """Constant wavenumber field of MP 2-A (§2): k^2 at every node."""
    return np.full((n + 1, n + 1), float(k) ** 2, dtype=np.float64)


def k2_from_velocity(c: np.ndarray, kh_max: float) -> np.ndarray:
    """k = 2 pi f / c with the frequency f chosen so that max(k) h = kh_max.

    The largest k sits where the velocity is smallest, so
    k = kh_max * n * c_min / c.
    """
    n = c.shape[0] - 1
    k = kh_max * n * float(c.min()) / c
    return (k * k).astype(np.float64)


def wedge_velocity(n: int, seed: int, c_top=2000.0, c_mid=1500.0, c_bot=3000.0) -> np.ndarray:
    """Three-layer wedge: interfaces y = 0.65 + s1 (x - 1/2), y = 0.35 + s2 (x - 1/2).

    Slopes s1, s2 ~ U(-0.2, 0.2) from the seed. Velocity c_top above the upper
    interface, c_mid between the interfaces and c_bot below the lower one.
    """
    rng = np.random.default_rng(seed)
    s1, s2 = rng.uniform(-0.2, 0.2, size=2)
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x, indexing="xy")  # [j, i]
    upper = 0.65 + s1 * (X - 0.5)
    lower = 0.35 + s2 * (X - 0.5)
    c = np.full((n + 1, n + 1), c_mid, dtype=np.float64)
    c[Y > upper] = c_top
    c[Y < lower] = c_bot
    return c


def _gaussian_filter_periodic(field: np.ndarray, sigma: float) -> np.ndarray:
    """Convolve with a unit-mass Gaussian of width sigma (unit coordinates), periodic."""
    m = field.shape[0]
    freq = np.fft.fftfreq(m, d=1.0 / m)  # integer wavenumbers on the unit period
    kx, ky = np.meshgrid(freq, freq, indexing="xy")
    transfer = np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx * kx + ky * ky))
    return np.real(np.fft.ifft2(np.fft.fft2(field) * transfer))


def grf_velocity(n: int, seed: int, corr: float = 0.1, c_min=1500.0, c_max=4500.0) -> np.ndarray:
    """Smooth Gaussian random velocity: N(0,1) white noise, Gaussian-filtered with
    correlation length `corr` (periodic FFT), mapped affinely onto [c_min, c_max]."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n + 1, n + 1))
    smooth = _gaussian_filter_periodic(noise, corr)
    lo, hi = smooth.min(), smooth.max()
    return c_min + (c_max - c_min) * (smooth - lo) / (hi - lo)


def smooth_k2(k2: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian-smoothed copy of a k^2 field (starting model of an inversion)."""
    return _gaussian_filter_periodic(k2, sigma)


def center_node(n: int) -> tuple[int, int]:
    """Node (i, j) at (1/2, 1/2), the source location of MP 2-A (§2)."""
    return (n // 2, n // 2)


def seeded_interior_nodes(n: int, count: int, seed: int) -> list[tuple[int, int]]:
    """`count` distinct interior nodes drawn from the seed."""
    rng = np.random.default_rng(seed)
    flat = rng.choice((n - 1) * (n - 1), size=count, replace=False)
    return [(int(f % (n - 1)) + 1, int(f // (n - 1)) + 1) for f in flat]


def top_row_sources(n: int, count: int) -> list[tuple[int, int]]:
    """Sources spread along the first interior row below the top edge."""
    return [(int(round((s + 0.5) * n / count)), n - 1) for s in range(count)]


def receiver_row(n: int, depth: float = 0.9) -> int:
    """Row index j of a horizontal receiver line at the given depth below the top."""
    return int(round((1.0 - depth) * n))


def point_source_rhs(n: int, nodes, amplitude=None) -> np.ndarray:
    """Right-hand side f of the PDE for unit point sources: 1/h^2 at each node.

    Returns complex128 of shape (len(nodes), n+1, n+1), one source per slice.
    """
    h = grid_h(n)
    amp = 1.0 / (h * h) if amplitude is None else amplitude
    f = np.zeros((len(nodes), n + 1, n + 1), dtype=np.complex128)
    for b, (i, j) in enumerate(nodes):
        f[b, j, i] = amp
    return f


def random_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded complex128 array with independent N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_k2(n: int, seed: int, k_lo: float, k_hi: float) -> np.ndarray:
    """Seeded k^2 field with k uniform in [k_lo, k_hi] node by node (rough profile)."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(k_lo, k_hi, size=(n + 1, n + 1))
    return k * k


def _unit_range(field: np.ndarray) -> np.ndarray:
    """Affine map of a field onto [0, 1] with both ends attained."""
    lo, hi = float(field.min()), float(field.max())
    chi = (field - lo) / (hi - lo)
    return np.clip(chi, 0.0, 1.0)


def chi_smooth(n: int, seed: int, corr: float = 0.1) -> np.ndarray:
    """MP 2-B medium-variation profile χ (§5.2, smooth changes): seeded N(0,1)
    white noise, Gaussian-filtered with width `corr` (periodic FFT), mapped onto
    [0, 1] so that the minimum is 0 and the maximum 1."""
    rng = np.random.default_rng(seed)
    return _unit_range(_gaussian_filter_periodic(rng.standard_normal((n + 1, n + 1)), corr))


def chi_sharp(n: int, seed: int) -> np.ndarray:
    """MP 2-B high-variation profile χ (§5.2, sharp changes): independent U(0, 1)
    values node by node, mapped onto [0, 1] so that both ends are attained."""
    rng = np.random.default_rng(seed)
    return _unit_range(rng.uniform(0.0, 1.0, size=(n + 1, n + 1)))


def k2_from_chi(chi: np.ndarray, k1: float, k2: float) -> np.ndarray:
    """k = k1 + (k2 - k1) χ of MP 2-B (§2), returned as k^2; k spans exactly
    [k1, k2] when χ spans [0, 1]."""
    k = float(k1) + (float(k2) - float(k1)) * chi
    return (k * k).astype(np.float64)


def mp2b_grid(k2: float, kh: float = 0.625) -> int:
    """Intervals n with max(k) h = kh (§2: the largest wavenumber obeys kh = 0.625)."""
    return int(round(float(k2) / kh))
