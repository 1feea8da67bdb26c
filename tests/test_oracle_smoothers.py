"""Pins of the oracle's smoothers: weighted Jacobi (paper §3) and GMRES(3) (§5.3)."""
import numpy as np
import scipy.sparse as sp

import oracle as O
from paper_2308_13476_amd import workloads as W


def test_jacobi_closed_form():
    A = sp.csr_matrix(np.array([[2 + 1j, 1.0], [1.0, 4.0]]))
    u = np.array([1.0 + 0j, 0.0])
    f = np.array([0.0 + 0j, 1.0])
    # r = f - A u = (-2 - i, 0); u + r / (4.5 (2 + i)) = (1 - 2/9, 0)
    np.testing.assert_allclose(O.jacobi_step(A, u, f, 4.5), [7.0 / 9.0, 0.0], atol=1e-15)


def test_omega_convention_optimal_for_poisson_is_three_halves():
    """With X = omega diag(A) the classical 1D Poisson smoothing optimum is omega = 3/2 (§3):
    the damping factor is 1/omega = 2/3. Brute force over omega on Fourier modes."""
    m = 64
    A = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1], format="lil")
    A[0, m - 1] = A[m - 1, 0] = -1.0  # periodic
    A = A.tocsr().astype(complex)
    j = np.arange(m)
    high = [2 * np.pi * q / m for q in range(m // 4, m // 2 + 1)]
    omegas = np.round(np.arange(1.0, 3.0, 0.01), 2)
    mu = []
    for om in omegas:
        amp = 0.0
        for t in high:
            v = np.exp(1j * t * j)
            out = O.jacobi_step(A, v, np.zeros(m, complex), om)
            amp = max(amp, np.abs(out).max())
        mu.append(amp)
    assert omegas[int(np.argmin(mu))] == 1.5


def test_gmres3_step_minimises_over_the_krylov_space():
    """Brute force: the new residual equals min over K_3(A, r0) computed by least squares on
    the explicit basis [A r0, A^2 r0, A^3 r0]; and it never grows."""
    n = 16
    k2 = W.random_k2(n, 7, 5.0, 20.0)
    H = O.build_hierarchy(k2, 1.0 / n, 0.1)
    A = H.A[0]
    rng = np.random.default_rng(8)
    u = W.random_complex((n + 1) ** 2, 9)
    f = W.random_complex((n + 1) ** 2, 10)
    r0 = f - A @ u
    K = np.stack([A @ r0, A @ (A @ r0), A @ (A @ (A @ r0))], axis=1)
    c = np.linalg.lstsq(K, r0, rcond=None)[0]
    best = np.linalg.norm(r0 - K @ c)
    u1 = O.gmres_step(A, u, f)
    got = np.linalg.norm(f - A @ u1)
    assert abs(got - best) <= 1e-10 * np.linalg.norm(r0)
    assert got <= np.linalg.norm(r0)
    # with the matching solution update: u1 = u + [r0, A r0, A^2 r0] c
    np.testing.assert_allclose(u1, u + np.stack([r0, A @ r0, A @ (A @ r0)], 1) @ c, rtol=0,
                               atol=1e-8 * np.abs(u1).max())
    del rng


def test_gmres_fp32_step_is_close_to_fp64():
    n = 16
    H = O.build_hierarchy(W.constant_k2(n, 6.0), 1.0 / n, 0.2)
    u = W.random_complex((n + 1) ** 2, 1)
    f = W.random_complex((n + 1) ** 2, 2)
    u64 = O.gmres_step(H.A[1 - 1], u, f)
    u32 = O.gmres_step(H.A32[0], u.astype(np.complex64), f.astype(np.complex64), breakdown=1e-6)
    assert u32.dtype == np.complex64
    assert np.linalg.norm(u32 - u64) / np.linalg.norm(u64) < 1e-4
