"""Two-grid diagnostics of §3.1 and §4.2 (oracle, CPU): the simplified
operator Gamma~, its HPD tests (Cholesky and the four element conditions)
and the optimality value ||Gamma~||_1 / kappa_1(Gamma~) of Table 2.
Pins: closed forms (D = A^{-1} gives Gamma = I; D = 0 gives 0),
T_0^H T_0 = I - Gamma against the separately built T_0, the HPD marks of
Table 1 (tests/golden/table1_two_grid_norms.json) where they are reproduced,
and the paper's corollary chain Gamma~ HPD => ||T_0||_2 < 1 on every case.
Table 2: evaluated on Gamma = I - T_0^H T_0 of the two-grid operator, 28 of
its 40 printed values are reproduced within 0.01 and all within 0.09 (on
Gamma~, the operator its caption names, they come out 0.4-0.9 of the printed
values)."""
import json
import os

import numpy as np
import pytest

from oracle import twogrid as TG

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_two_grid_norms.json")


def test_gamma_closed_forms():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)) + 6 * np.eye(12)
    np.testing.assert_allclose(TG.gamma_of(A, np.linalg.inv(A)), np.eye(12), atol=1e-12)
    np.testing.assert_allclose(TG.gamma_of(A, np.zeros_like(A)), np.zeros((12, 12)))
    # D = c A^{-1}: D A = c I, Gamma = (2c - c^2) I
    np.testing.assert_allclose(TG.gamma_of(A, 0.5 * np.linalg.inv(A)), 0.75 * np.eye(12), atol=1e-12)


@pytest.mark.parametrize("nu", [1, 2])
def test_gamma_equals_identity_minus_t0h_t0(nu):
    # the same D = I - T_0 A^{-1}, with T_0 built from the smoother and the coarse correction
    A, M, Q = TG.two_grid_parts(10, 16, nu=nu)
    T0 = TG.two_grid_operator(10, 16, nu=nu)
    D = (np.eye(A.shape[0]) - T0) @ np.linalg.inv(A)
    G = TG.gamma_of(A, D)
    np.testing.assert_allclose(G, np.eye(A.shape[0]) - T0.conj().T @ T0, atol=1e-9)
    assert np.linalg.norm(G - G.conj().T) < 1e-9


def test_gamma_tilde_is_hermitian_and_drops_only_the_cross_term():
    A, M, Q = TG.two_grid_parts(5, 8)
    Gt = TG.gamma_tilde(5, 8)
    assert np.linalg.norm(Gt - Gt.conj().T) < 1e-10 * np.linalg.norm(Gt)
    # one Jacobi step: M = X^{-1} with X = omega diag(A)
    np.testing.assert_allclose(M, np.diag(1.0 / (4.5 * np.diag(A))), atol=1e-12)


def test_hpd_tests_agree_on_constructed_matrices():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
    H = B @ B.conj().T + 0.1 * np.eye(10)
    assert TG.is_hpd_cholesky(H) and all(TG.hpd_conditions(H).values())
    neg = H.copy()
    neg[3, 3] = -1.0  # negative diagonal entry: not HPD, first condition fails
    assert not TG.is_hpd_cholesky(neg) and not TG.hpd_conditions(neg)["positive_diagonal"]
    big = np.eye(4, dtype=complex)
    big[0, 1] = big[1, 0] = 3.0  # off-diagonal larger than the diagonal
    assert not TG.is_hpd_cholesky(big)
    c = TG.hpd_conditions(big)
    assert not c["pairs"] and not c["max_on_diagonal"] and not c["positive_determinant"]
    assert not TG.is_hpd_cholesky(rng.standard_normal((5, 5)))  # not Hermitian


def test_table1_hpd_marks_where_reproduced():
    g = json.load(open(GOLDEN))
    cols = {"linear_A": ("linear", "A"), "linear_C": ("linear", "C"), "bezier_A": ("bezier", "A"),
            "bezier_C": ("bezier", "C")}
    got = {c: [TG.is_hpd_cholesky(TG.gamma_tilde(k, n, transfer=t, coarse_on=o)) for k, n in zip(g["k"], g["n"])]
           for c, (t, o) in cols.items()}
    agree = sum(a == b for c in cols for a, b in zip(got[c], g["gamma_tilde_hpd"][c]))
    assert agree >= 14, got  # 14 of the 16 marks; the design notes name the two that differ
    assert got["linear_A"] == got["linear_C"] == [False] * 4
    assert got["bezier_C"][:3] == [True, True, True]


@pytest.mark.parametrize("transfer,coarse_on", [("bezier", "C"), ("bezier", "A"), ("linear", "C")])
@pytest.mark.parametrize("omega,nu", [(1.5, 1), (4.5, 1), (4.5, 2), (7.0, 2)])
def test_corollary_chain_gamma_tilde_hpd_implies_convergent_two_grid(transfer, coarse_on, omega, nu):
    for k, n in [(5, 8), (10, 16)]:
        Gt = TG.gamma_tilde(k, n, transfer=transfer, coarse_on=coarse_on, omega=omega, nu=nu)
        T0 = TG.two_grid_operator(k, n, transfer=transfer, coarse_on=coarse_on, omega=omega, nu=nu)
        if TG.is_hpd_cholesky(Gt):
            assert np.linalg.norm(T0, 2) < 1.0
            assert 0.0 < TG.optimality_value(Gt) <= 1.0


def test_table2_trends_at_omega_4_5():
    # Table 2 at omega = 4.5: a second smoothing step raises the value at every
    # k, and the value falls as k grows; both hold for the oracle's values
    # (the values themselves are 0.4-0.9 of the printed ones: unpinned).
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table2_optimality.json")))
    q = g["omega"].index(4.5)
    paper1, paper2 = g["values_nu1"][q], g["values_nu2"][q]
    v1 = [TG.optimality_value(TG.gamma_tilde(k, n, omega=4.5, nu=1)) for k, n in zip(g["k"], g["n"])]
    v2 = [TG.optimality_value(TG.gamma_tilde(k, n, omega=4.5, nu=2)) for k, n in zip(g["k"], g["n"])]
    for vals in (paper1, paper2, v1, v2):
        assert all(a > b for a, b in zip(vals, vals[1:]))
    assert all(b > a for a, b in zip(paper1, paper2)) and all(b > a for a, b in zip(v1, v2))


def test_optimality_value_against_explicit_norms_and_a_hand_worked_case():
    # ||B||_1 / kappa_1(B) with kappa_1 = ||B||_1 ||B^{-1}||_1 from an explicit
    # inverse (column sums of moduli), on a Hermitian positive definite matrix
    rng = np.random.default_rng(11)
    Z = rng.standard_normal((9, 9)) + 1j * rng.standard_normal((9, 9))
    B = Z @ Z.conj().T + 0.5 * np.eye(9)
    Binv = np.linalg.inv(B)
    n1 = np.abs(B).sum(axis=0).max()
    kappa = n1 * np.abs(Binv).sum(axis=0).max()
    assert TG.optimality_value(B) == pytest.approx(n1 / kappa, rel=1e-12)
    # by hand: B = [[2, i], [-i, 2]] has B^{-1} = [[2, -i], [i, 2]] / 3, so
    # ||B||_1 = 3, ||B^{-1}||_1 = 1, kappa_1 = 3 and the value is 3 / 3 = 1
    B2 = np.array([[2.0, 1j], [-1j, 2.0]])
    assert TG.optimality_value(B2) == pytest.approx(1.0, rel=1e-14)
    # diag(1, 4): ||B||_1 = 4, kappa_1 = 4, value 1 = the smallest eigenvalue
    assert TG.optimality_value(np.diag([1.0, 4.0])) == pytest.approx(1.0, rel=1e-14)


def test_two_smoothing_steps_give_the_expanded_approximate_inverse():
    # nu = 2: (I - S^2) A^{-1} with S = I - X^{-1} A expands to
    # 2 X^{-1} - X^{-1} A X^{-1}, which needs no inverse of A
    A, M, Q = TG.two_grid_parts(5, 8, nu=2, omega=4.5)
    Xi = np.diag(1.0 / (4.5 * np.diag(A)))
    np.testing.assert_allclose(M, 2 * Xi - Xi @ A @ Xi, atol=1e-12 * np.abs(M).max())
    # the coarse part is a projection-like map: Q A Q = Q when A_c = R A P
    A2, M2, Q2 = TG.two_grid_parts(5, 8, coarse_on="A")
    np.testing.assert_allclose(Q2 @ A2 @ Q2, Q2, atol=1e-9 * np.abs(Q2).max())


def test_table2_values_on_the_two_grid_gamma():
    """§4.2 Table 2 (omega in {1.5, 2, 2.5, 4.5, 7}, nu in {1, 2}, k in
    {5, 10, 20, 30} at kh = 0.625) against the printed values: the omega = 4.5
    column that the experiments use within 0.006 (nu = 1) and 0.02 (nu = 2),
    28 of the 40 entries within 0.01 (35 within 0.02), every entry within 0.09; and the paper's
    reading of the table: at omega = 4.5 a second smoothing step raises the
    value at every k, at omega = 1.5 it lowers it for k >= 20."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table2_optimality.json")))
    within = 0
    got = {}
    for q, om in enumerate(g["omega"]):
        for nu, key in ((1, "values_nu1"), (2, "values_nu2")):
            vals = [TG.table2_value(k, n, om, nu) for k, n in zip(g["k"], g["n"])]
            got[om, nu] = vals
            err = [abs(a - b) for a, b in zip(vals, g[key][q])]
            assert max(err) <= 0.09, (om, nu, vals, g[key][q])
            within += sum(e <= 0.01 for e in err)
            if om == 4.5:
                assert max(err) <= (0.006 if nu == 1 else 0.02), (nu, vals, g[key][q])
    assert within >= 28, within
    assert all(b > a for a, b in zip(got[4.5, 1], got[4.5, 2]))
    assert all(b < a for a, b in zip(got[1.5, 1][2:], got[1.5, 2][2:]))
    # the simplified operator of the caption gives markedly smaller values
    k, n = g["k"][0], g["n"][0]
    assert TG.table2_value(k, n, 4.5, 1, operator="gamma_tilde") < 0.5 * got[4.5, 1][0]
