"""Pins of the oracle's stiffness form with a constant symmetric diffusion
matrix A (Example 1's A; the diffusion is a(x) A): K[m][n] = sum_x w a |det J|
(J^-T grad phi_n) . A (J^-T grad phi_m).  Each check fixes the form by
something other than the oracle itself."""
import numpy as np
import pytest

import oracle
from paper_1809_05471_amd import inputs
from tests.bruteforce import dense_bruteforce
from tests.test_oracle_pins import _onedim_matrices

A2 = np.array([[1.3, 0.4], [0.4, 0.7]])
A3 = np.array([[1.2, 0.3, -0.2], [0.3, 0.9, 0.25], [-0.2, 0.25, 1.6]])


@pytest.mark.parametrize("S", [np.array([[1.0, 0.3], [0.2, 1.1]]), np.array([[0.8, -0.5], [0.4, 1.2]])])
def test_affine_map_2d(S):
    """G(xhat) = S xhat: C = |det S| S^-1 A S^-T in the Kronecker form of the
    1D matrices (scipy tables); S^-T A S^-1 in its place fails."""
    K, p = (4, 3), 3
    kn, ctrl0 = inputs.identity_geometry(K, p)
    P = oracle.Problem(kn, p, ctrl0 @ S.T, diff_A=A2)
    Si = np.linalg.inv(S)
    C = abs(np.linalg.det(S)) * Si @ A2 @ Si.T
    assert np.abs(C - abs(np.linalg.det(S)) * Si.T @ A2 @ Si).max() > 1e-2
    m1, s1, x1 = _onedim_matrices(kn[0], p)
    m2, s2, x2 = _onedim_matrices(kn[1], p)
    Kexp = (C[0, 0] * np.kron(m2, s1) + C[0, 1] * np.kron(x2.T, x1) + C[1, 0] * np.kron(x2, x1.T)
            + C[1, 1] * np.kron(s2, m1))
    assert np.abs(P.dense(oracle.STIFF) - Kexp).max() < 1e-13 * np.abs(Kexp).max()


@pytest.mark.parametrize("K,p", [((4, 5), 2), ((5, 4), 3)])
def test_patch_test_2d(K, p):
    """u = gamma . x has a constant gradient, so div(A grad u) = 0 and
    (K x)_m vanishes on interior rows in any geometry (exact quadrature in
    d = 2)."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=11, amp=0.3)
    P = oracle.Problem(kn, p, ctrl, diff_A=A2)
    x = ctrl @ np.array([0.7, -1.3])
    y = P.dense(oracle.STIFF) @ x
    n1, n2 = K[0] + p - 1, K[1] + p - 1
    idx = np.arange(P.N)
    i1, i2 = idx % n1, idx // n1
    interior = (i1 > 0) & (i1 < n1 - 1) & (i2 > 0) & (i2 < n2 - 1)
    assert np.abs(y[interior]).max() < 1e-12 * np.abs(x).max()
    assert np.abs(y[~interior]).max() > 1e-3


@pytest.mark.parametrize("d,K,p,coef", [(2, (3, 4), 2, ("sinprod", 0.5)), (3, (2, 3, 2), 3, ("sinprod", 0.5)),
                                        (3, (2, 2, 2), 4, ("const", 1.5))])
def test_dense_bruteforce_algebraic_form(d, K, p, coef):
    A = A2 if d == 2 else A3
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=13, amp=0.2)
    P = oracle.Problem(kn, p, ctrl, coef, diff_A=A)
    Kd = P.dense(oracle.STIFF)
    B = dense_bruteforce(kn, p, ctrl, coef, 2, diff_A=A)
    assert np.abs(Kd - B).max() <= 1e-13 * np.abs(B).max()
    assert np.abs(Kd - Kd.T).max() <= 1e-13 * np.abs(Kd).max()


def test_identity_matrix_is_the_default():
    kn, ctrl = inputs.perturbed_geometry((2, 3, 2), 3, seed=3, amp=0.2)
    a = oracle.Problem(kn, 3, ctrl, ("sinprod", 0.5)).dense(oracle.STIFF)
    b = oracle.Problem(kn, 3, ctrl, ("sinprod", 0.5), diff_A=np.eye(3)).dense(oracle.STIFF)
    assert np.array_equal(a, b)
