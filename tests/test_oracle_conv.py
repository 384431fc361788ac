"""Pins of the oracle's convection form (op 4): the b . grad u term of the
convection-diffusion equation (Sec. 2, Example 1) tested with v, entry
B[m][n] = sum_x w s(G) |det J| (b . J^-T grad phi_n) phi_m.

Each check fixes the form by something other than the oracle itself:
integration by parts in 1D (exact under the p-point Gauss rule), the
Kronecker structure on the identity and affine maps from scipy's B-spline
tables, the exact image of the coordinate function x_1 on curved maps, and
the dense algebraic form of Sec. 5 built with numpy.linalg."""
import numpy as np
import pytest

import oracle
from paper_1809_05471_amd import inputs
from tests.bruteforce import basis_1d, dense_bruteforce, gauss_points_1d


def _onedim(kn, p):
    x, w = gauss_points_1d(kn, p)
    V, D = basis_1d(kn, p, x)
    mass = V.T @ (w[:, None] * V)
    grad = V.T @ (w[:, None] * D)          # grad[m, n] = int phi_n' phi_m
    return mass, grad


@pytest.mark.parametrize("K,p", [(5, 2), (7, 3), (4, 5), (3, 9)])
def test_1d_integration_by_parts(K, p):
    """Identity map, b = 1: B + B^T = e_N e_N^T - e_1 e_1^T (open knots: only
    the first and last functions are nonzero at the ends, where they are 1);
    Gauss with p points integrates phi_n' phi_m (degree 2p - 3) exactly."""
    kn, ctrl = inputs.identity_geometry((K,), p)
    P = oracle.Problem(kn, p, ctrl, conv_b=(1.0,))
    B = P.dense(oracle.CONV)
    n = B.shape[0]
    E = np.zeros((n, n))
    E[0, 0], E[-1, -1] = -1.0, 1.0
    assert np.abs(B + B.T - E).max() < 1e-14
    assert np.abs(B - B.T).max() > 0.1                     # not symmetric
    assert np.abs(B.sum(axis=1)).max() < 1e-14             # grad of the constant 1


@pytest.mark.parametrize("K,p", [((3, 4, 2), 2), ((3, 2, 3), 3), ((2, 2, 2), 4)])
def test_identity_map_is_kronecker(K, p):
    """Identity map, constant b: B = sum_k b_k kron(.., G_k in slot k, ..)
    with the 1D mass M and G[m, n] = int phi_n' phi_m from scipy tables
    (lexicographic, direction 1 fastest).  A swapped trial/test side gives
    G^T in the slot and fails."""
    b = (0.7, -1.3, 0.4)
    kn, ctrl = inputs.identity_geometry(K, p)
    P = oracle.Problem(kn, p, ctrl, coef=("const", 1.5), conv_b=b)
    one = [_onedim(kn[k], p) for k in range(3)]

    def kron(mats):
        out = mats[-1]
        for m in mats[-2::-1]:
            out = np.kron(out, m)
        return out

    exp = 1.5 * sum(b[j] * kron([one[k][1] if k == j else one[k][0] for k in range(3)]) for j in range(3))
    assert np.abs(P.dense(oracle.CONV) - exp).max() < 1e-14 * np.abs(exp).max() * 10


@pytest.mark.parametrize("S", [np.array([[1.0, 0.3], [0.2, 1.1]]), np.array([[0.8, -0.5], [0.4, 1.2]])])
def test_affine_map_2d(S):
    """G(xhat) = S xhat: b . J^-T grad_hat = (S^-1 b) . grad_hat, so
    B = |det S| sum_k (S^-1 b)_k kron(.., G_k in slot k, ..).  J^-T b in its
    place fails for these non-symmetric S."""
    K, p = (4, 3), 3
    b = np.array([0.6, -0.9])
    kn, ctrl0 = inputs.identity_geometry(K, p)
    ctrl = ctrl0 @ S.T
    P = oracle.Problem(kn, p, ctrl, conv_b=b)
    v = np.linalg.solve(S, b)
    assert np.abs(v - np.linalg.solve(S.T, b)).max() > 1e-2
    m1, g1 = _onedim(kn[0], p)
    m2, g2 = _onedim(kn[1], p)
    exp = abs(np.linalg.det(S)) * (v[0] * np.kron(m2, g1) + v[1] * np.kron(g2, m1))
    assert np.abs(P.dense(oracle.CONV) - exp).max() < 1e-13 * np.abs(exp).max()


@pytest.mark.parametrize("d,K,p,coef", [
    (2, (4, 3), 3, ("const", 1.7)),
    (3, (3, 2, 3), 2, ("const", 0.8)),
    (3, (2, 3, 2), 4, ("const", 1.2)),
])
def test_coordinate_function_on_curved_maps(d, K, p, coef):
    """u = x_i, the physical coordinate, has coefficients ctrl[:, i] (G =
    sum c_n phi_n) and J^-T grad_hat u = e_i exactly at every point, so
    B ctrl[:, i] = s b_i M 1 on any map (M the mass matrix, c = 1, and s the
    constant coefficient); and B 1 = 0 (partition of unity).  A J^-1 in
    place of J^-T breaks the first on these curved maps."""
    b = (0.5, -1.1, 0.9)[:d]
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=5, amp=0.2)
    P = oracle.Problem(kn, p, ctrl, coef=coef, conv_b=b)
    B = P.dense(oracle.CONV)
    M1 = P.dense(oracle.MASS) @ np.ones(P.N)
    for i in range(d):
        exp = coef[1] * b[i] * M1
        assert np.abs(B @ ctrl[:, i] - exp).max() < 1e-13 * np.abs(M1).max()
    assert np.abs(B @ np.ones(P.N)).max() < 1e-13 * np.abs(B).max()


@pytest.mark.parametrize("d,K,p,coef", [
    (2, (3, 4), 2, ("sinprod", 0.5)),
    (3, (2, 3, 2), 3, ("sinprod", 0.5)),
    (3, (2, 2, 2), 4, ("const", 1.5)),
])
def test_dense_bruteforce_algebraic_form(d, K, p, coef):
    """Oracle == dense Q_Psi^T F Q_Phi (Sec. 5) with the convection block of
    F, from scipy tables and numpy.linalg, on tiny perturbed meshes."""
    b = (0.3, -0.8, 1.1)[:d]
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=13, amp=0.2)
    P = oracle.Problem(kn, p, ctrl, coef, conv_b=b)
    A = P.dense(oracle.CONV)
    B = dense_bruteforce(kn, p, ctrl, coef, 4, conv_b=b)
    assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


def test_rows_and_apply_agree_with_full_assembly():
    """The row, apply and per-element paths of op 4 equal the full matrix."""
    K, p = (3, 4, 3), 3
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=2)
    P = oracle.Problem(kn, p, ctrl, ("sinprod", 0.5), conv_b=(0.4, 1.0, -0.6))
    A = P.dense(oracle.CONV)
    x = inputs.random_vector(P.N, seed=3)
    y = A @ x
    assert np.abs(P.apply(oracle.CONV, x) - y).max() < 1e-13 * np.abs(y).max()
    rows = np.array([0, 5, P.N // 2, P.N - 1])
    assert np.abs(P.apply_rows(oracle.CONV, x, rows) - y[rows]).max() < 1e-13 * np.abs(y).max()
    assert np.abs(P.apply_rows_by_elements(oracle.CONV, x, rows) - y[rows]).max() < 1e-13 * np.abs(y).max()
    for m, (cols, vals) in zip(rows, P.rows(oracle.CONV, rows)):
        assert np.abs(A[m, cols] - vals).max() < 1e-15 * np.abs(A).max() * 10
