"""Pins of the oracle against facts the paper and the mathematics fix.

Each test checks the oracle (``oracle/``) against something other than
itself: library routines (scipy BSpline, Gauss exactness), closed forms
(cardinal and Bernstein Gram matrices), invariants (symmetry, partition of
unity, domain measure by Green's theorem, patch test), affine maps with a
known answer, the exact #NZ count for open knot vectors (Corollary in Sec.
3.2), and a dense brute force of the algebraic form of Sec. 5.
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

import oracle
from paper_1809_05471_amd import inputs
from tests.bruteforce import basis_1d, dense_bruteforce, gauss_points_1d

pytestmark = pytest.mark.filterwarnings("ignore")


def _nonuniform_knots(p):
    inner = [0.1, 0.25, 0.25, 0.6, 0.85] if p >= 3 else [0.1, 0.25, 0.6, 0.85]
    return np.array([0.0] * p + inner + [1.0] * p)


# ---------------------------------------------------------------- 1D tables

@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("uniform", [True, False])
def test_tables_match_scipy_bspline(p, uniform):
    """Cox-de Boor tables equal scipy's B-spline evaluator (values and derivatives)."""
    kn = inputs.open_uniform_knots(5, p) if uniform else _nonuniform_knots(p)
    if p == 1 and not uniform:
        kn = np.array([0.0, 0.1, 0.25, 0.6, 0.85, 1.0])
    T = oracle.tables_1d(kn, p)
    x = T["x"].ravel()
    V, D = basis_1d(kn, p, x)
    for e in range(T["nel"]):
        for g in range(p):
            row = e * p + g
            for j in range(p):
                n = T["first"][e] + j
                assert abs(T["phi"][e, g, j] - V[row, n]) < 1e-14
                assert abs(T["dphi"][e, g, j] - D[row, n]) < 1e-11 * max(1.0, abs(D[row, n]))
            # every function not listed as active is zero at this point
            inactive = np.ones(T["nfun"], bool)
            inactive[T["first"][e]:T["first"][e] + p] = False
            assert np.all(V[row, inactive] == 0.0)


@pytest.mark.parametrize("p", [2, 3, 4, 6, 9])
def test_partition_of_unity(p):
    T = oracle.tables_1d(_nonuniform_knots(p), p)
    assert np.allclose(T["phi"].sum(axis=2), 1.0, atol=1e-14)
    assert np.allclose(T["dphi"].sum(axis=2), 0.0, atol=1e-11)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 9])
def test_gauss_rule_exactness(p):
    """p-point Gauss on every element integrates degree 2p-1 exactly, not 2p."""
    kn = _nonuniform_knots(max(p, 2)) if p > 1 else np.array([0.0, 0.3, 1.0])
    T = oracle.tables_1d(kn, p)
    x, w = T["x"], T["w"]
    assert abs(w.sum() - 1.0) < 1e-14
    for k in range(2 * p):
        exact = 1.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-13
    # one element on [0, 1]: degree 2p is no longer integrated exactly
    T1 = oracle.tables_1d(inputs.open_uniform_knots(1, p), p)
    assert abs((T1["w"] * T1["x"] ** (2 * p)).sum() - 1.0 / (2 * p + 1)) > 1e-14


# ------------------------------------------------------ 1D closed forms

def _cardinal(m, x, deriv=0):
    """Cardinal B-spline of order m on [0, m] (or its derivative) at rational x
    from the truncated-power representation."""
    x = Fraction(x)
    s = Fraction(0)
    pw = m - 1 - deriv
    for j in range(m + 1):
        u = x - j
        if u > 0:
            s += (-1) ** j * comb(m, j) * u ** pw
    return s / factorial(pw)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_interior_rows_cardinal_closed_form(p):
    """Interior rows of the 1D uniform mass/stiffness matrices:
    int N_p(x) N_p(x-k) = N_2p(p+k) and int N_p' N_p'(.-k) = -N_2p''(p+k)."""
    K = 2 * p + 3
    kn, ctrl = inputs.identity_geometry((K,), p)
    P = oracle.Problem(kn, p, ctrl)
    M = P.dense(oracle.MASS)
    S = P.dense(oracle.STIFF)
    h = 1.0 / K
    m = (K + p - 1) // 2          # support entirely interior
    for k in range(-(p - 1), p):
        em = float(_cardinal(2 * p, p + k))
        es = float(-_cardinal(2 * p, p + k, deriv=2))
        assert abs(M[m, m + k] / h - em) < 1e-14
        assert abs(S[m, m + k] * h - es) < 1e-12
    assert np.all(M[m, m + p:] == 0) and np.all(M[m, :m - p + 1] == 0)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 7, 9])
def test_single_element_bernstein_closed_form(p):
    """K = 1: the B-splines are the Bernstein polynomials of degree q = p-1;
    Gram matrix C(q,i)C(q,j)/(C(2q,i+j)(2q+1)) and, via
    B'_{i,q} = q(B_{i-1,q-1} - B_{i,q-1}), the stiffness matrix."""
    q = p - 1
    kn, ctrl = inputs.identity_geometry((1,), p)
    P = oracle.Problem(kn, p, ctrl)
    M = P.dense(oracle.MASS)
    S = P.dense(oracle.STIFF)

    def gram(deg, i, j):
        if i < 0 or j < 0 or i > deg or j > deg:
            return Fraction(0)
        return Fraction(comb(deg, i) * comb(deg, j), comb(2 * deg, i + j) * (2 * deg + 1))

    for i in range(p):
        for j in range(p):
            assert abs(M[i, j] - float(gram(q, i, j))) < 1e-15
            s = q * q * (gram(q - 1, i - 1, j - 1) - gram(q - 1, i - 1, j)
                         - gram(q - 1, i, j - 1) + gram(q - 1, i, j))
            assert abs(S[i, j] - float(s)) < 1e-12 * max(1, abs(float(s)))


# --------------------------------------------------------- tensor structure

@pytest.mark.parametrize("d,K,p", [(2, (4, 3), 2), (2, (5, 4), 3), (3, (3, 2, 4), 2), (3, (3, 3, 2), 3)])
def test_identity_geometry_is_kronecker(d, K, p):
    """Identity map: M = kron of 1D mass matrices, K = sum over directions of
    kron with the 1D stiffness in that slot (lexicographic, direction 1 fastest)."""
    kn, ctrl = inputs.identity_geometry(K, p)
    P = oracle.Problem(kn, p, ctrl)
    M1, S1 = [], []
    for k in range(d):
        kk, cc = inputs.identity_geometry((K[k],), p)
        Q = oracle.Problem(kk, p, cc)
        M1.append(Q.dense(oracle.MASS))
        S1.append(Q.dense(oracle.STIFF))

    def kron(mats):
        out = mats[-1]
        for m in mats[-2::-1]:
            out = np.kron(out, m)
        return out

    Mexp = kron(M1)
    Sexp = sum(kron([S1[k] if k == j else M1[k] for k in range(d)]) for j in range(d))
    assert np.abs(P.dense(oracle.MASS) - Mexp).max() < 1e-15
    assert np.abs(P.dense(oracle.STIFF) - Sexp).max() < 1e-13


@pytest.mark.parametrize("d,K,p", [(1, (7,), 3), (2, (5, 6), 2), (2, (4, 4), 4), (3, (3, 4, 5), 3)])
def test_nnz_matches_corollary(d, K, p):
    """#NZ = prod_delta (q N + p M - sum mu mu) = prod (N (2p-1) - p (p-1))."""
    kn, ctrl = inputs.identity_geometry(K, p)
    P = oracle.Problem(kn, p, ctrl)
    rp, ci = P.pattern()
    exp = 1
    for k in K:
        n = k + p - 1
        exp *= n * (2 * p - 1) - p * (p - 1)
    assert rp[-1] == exp
    # columns ascending and within the band of every row
    for m in range(P.N):
        c = ci[rp[m]:rp[m + 1]]
        assert np.all(np.diff(c) > 0)


def test_nnz_nonuniform_multiplicity():
    """Open knots with a double interior knot: exact #NZ per the Corollary."""
    p = 3
    kn = _nonuniform_knots(p)                       # 0.25 has multiplicity 2
    T = oracle.tables_1d(kn, p)
    P = oracle.Problem([kn], p, np.linspace(0, 1, T["nfun"])[:, None] ** 1)
    rp, _ = P.pattern()
    N = T["nfun"]
    # sum over distinct knots except the last of mu^2: 0 -> p, interior simple -> 1, double -> 4
    mu = [p, 1, 2, 1, 1]
    assert rp[-1] == 2 * p * N - sum(m * m for m in mu)


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("d,K,p", [(2, (5, 4), 3), (3, (3, 3, 4), 2), (3, (2, 3, 2), 4)])
def test_symmetry_and_row_sums(d, K, p):
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=7)
    P = oracle.Problem(kn, p, ctrl, ("sinprod", 0.5))
    S = P.dense(oracle.STIFF)
    M = P.dense(oracle.MASS)
    scale = np.abs(S).max()
    assert np.abs(S - S.T).max() <= 1e-14 * scale
    assert np.abs(M - M.T).max() <= 1e-15
    assert np.abs(S.sum(axis=1)).max() <= 1e-13 * scale       # K 1 = 0
    assert np.all(np.diag(S) > 0) and np.all(np.diag(M) > 0)


def _boundary_area_2d(knots, p, ctrl, K):
    """Area of the image of [0,1]^2 from its four boundary spline curves by
    Green's theorem (1/2) ∮ (x dy - y dx), scipy BSpline curves and high-order
    Gauss per knot span (exact for the polynomial integrand)."""
    from scipy.interpolate import BSpline
    n1, n2 = K[0] + p - 1, K[1] + p - 1
    C = ctrl.reshape(n2, n1, 2)
    curves = [(knots[0], C[0, :, :], False), (knots[1], C[:, -1, :], False),
              (knots[0], C[-1, :, :], True), (knots[1], C[:, 0, :], True)]
    area = 0.0
    nodes, weights = np.polynomial.legendre.leggauss(2 * p + 2)
    for kn, cp, rev in curves:
        spl = BSpline(kn, cp, p - 1)
        der = spl.derivative()
        br = np.unique(kn)
        for a, b in zip(br[:-1], br[1:]):
            s = a + (b - a) * (nodes + 1) / 2
            ws = weights * (b - a) / 2
            xy, dxy = spl(s), der(s)
            contrib = 0.5 * np.sum(ws * (xy[:, 0] * dxy[:, 1] - xy[:, 1] * dxy[:, 0]))
            area += -contrib if rev else contrib
    return area


@pytest.mark.parametrize("K,p", [((4, 5), 2), ((3, 4), 3), ((5, 3), 4), ((2, 2), 6)])
def test_mass_sum_equals_domain_area_2d(K, p):
    """1^T M 1 = sum_x w |det J| = area of G([0,1]^2): exact in d = 2 since
    det J has degree <= 2p-3 per direction (p Gauss points integrate 2p-1)."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=3, amp=0.2)
    P = oracle.Problem(kn, p, ctrl)
    M = P.dense(oracle.MASS)
    area = _boundary_area_2d(kn, p, ctrl, K)
    assert abs(M.sum() - area) < 1e-13
    assert abs(P.measure() - area) < 1e-13
    assert abs(area - 1.0) > 1e-6        # the boundary really moved


@pytest.mark.parametrize("K,p", [((3, 3, 3), 2), ((3, 2, 3), 3)])
def test_mass_sum_unit_volume_3d_interior_perturbation(K, p):
    """Interior-only perturbation keeps the boundary, so the volume is 1; for
    p <= 3, det J (degree <= 3p-4 per direction) is integrated exactly."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=5, amp=0.3, interior_only=True)
    P = oracle.Problem(kn, p, ctrl)
    assert abs(P.dense(oracle.MASS).sum() - 1.0) < 1e-14


@pytest.mark.parametrize("K,p", [((4, 5), 2), ((4, 4), 3), ((3, 5), 4)])
def test_patch_test_2d(K, p):
    """u = gamma . x is exactly represented by x_n = gamma . c_n; then
    (K x)_m = ∮ gamma.n phi_m = 0 for interior rows m, and in d = 2 the
    quadrature is exact (integrand cof(J) grad phi_m has degree <= 2p-2).
    Fails if J and J^T are swapped in the pull-back."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=11, amp=0.3)
    P = oracle.Problem(kn, p, ctrl)
    gamma = np.array([0.7, -1.3])
    x = ctrl @ gamma
    y = P.dense(oracle.STIFF) @ x
    n1, n2 = K[0] + p - 1, K[1] + p - 1
    idx = np.arange(P.N)
    i1, i2 = idx % n1, idx // n1
    interior = (i1 > 0) & (i1 < n1 - 1) & (i2 > 0) & (i2 < n2 - 1)
    assert np.abs(y[interior]).max() < 1e-12 * np.abs(x).max()
    assert np.abs(y[~interior]).max() > 1e-3           # boundary rows carry the flux


def _onedim_matrices(kn, p):
    x, w = gauss_points_1d(kn, p)
    V, D = basis_1d(kn, p, x)
    mass = V.T @ (w[:, None] * V)
    stiff = D.T @ (w[:, None] * D)
    mix = D.T @ (w[:, None] * V)          # mix[m, n] = int phi_m' phi_n
    return mass, stiff, mix


@pytest.mark.parametrize("S", [np.array([[1.0, 0.3], [0.2, 1.1]]), np.array([[0.8, -0.5], [0.4, 1.2]])])
def test_affine_map_2d(S):
    """G(xhat) = S xhat: J = S, C = |det S| S^-1 S^-T; K = sum_ij C_ij
    int d_i phi_m d_j phi_n assembled from 1D matrices (scipy tables).  A
    swapped transpose (S^-T S^-1) fails for these non-normal S."""
    K, p = (4, 3), 3
    kn, ctrl0 = inputs.identity_geometry(K, p)
    ctrl = ctrl0 @ S.T
    P = oracle.Problem(kn, p, ctrl)
    Sinv = np.linalg.inv(S)
    C = abs(np.linalg.det(S)) * Sinv @ Sinv.T
    assert np.abs(Sinv @ Sinv.T - Sinv.T @ Sinv).max() > 1e-2
    m1, s1, x1 = _onedim_matrices(kn[0], p)
    m2, s2, x2 = _onedim_matrices(kn[1], p)
    # matrices on the 2D lexicographic index: kron(direction 2, direction 1)
    T11 = np.kron(m2, s1)
    T22 = np.kron(s2, m1)
    T12 = np.kron(x2.T, x1)               # d_1 on test, d_2 on trial
    T21 = np.kron(x2, x1.T)
    Kexp = C[0, 0] * T11 + C[0, 1] * T12 + C[1, 0] * T21 + C[1, 1] * T22
    assert np.abs(P.dense(oracle.STIFF) - Kexp).max() < 1e-13 * np.abs(Kexp).max()
    Mexp = abs(np.linalg.det(S)) * np.kron(m2, m1)
    assert np.abs(P.dense(oracle.MASS) - Mexp).max() < 1e-15


@pytest.mark.parametrize("d,K,p,coef", [
    (1, (5,), 3, ("const", 2.0)),
    (2, (3, 4), 2, ("sinprod", 0.5)),
    (2, (2, 3), 4, ("sinprod", 0.9)),
    (3, (2, 3, 2), 3, ("sinprod", 0.5)),
    (3, (2, 2, 2), 4, ("const", 1.5)),
])
def test_dense_bruteforce_algebraic_form(d, K, p, coef):
    """Oracle == dense Q_Psi^T F Q_Phi (Sec. 5) on tiny perturbed meshes."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=13, amp=0.2)
    P = oracle.Problem(kn, p, ctrl, coef)
    for op in (oracle.MASS, oracle.STIFF):
        A = P.dense(op)
        B = dense_bruteforce(kn, p, ctrl, coef, op)
        assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


# ------------------------------------------------------------ oracle paths

def test_rows_and_apply_agree_with_full_assembly():
    K, p = (3, 4, 3), 3
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=2)
    P = oracle.Problem(kn, p, ctrl, ("sinprod", 0.5))
    x = inputs.random_vector(P.N, 0)
    for op in (oracle.MASS, oracle.STIFF):
        rp, ci, v = P.assemble(op)
        rows = np.array([0, 5, P.N // 2, P.N - 1])
        got = P.rows(op, rows)
        for r, (c, vals) in zip(rows, got):
            assert np.array_equal(c, ci[rp[r]:rp[r + 1]])
            assert np.abs(vals - v[rp[r]:rp[r + 1]]).max() < 1e-14 * np.abs(v).max()
        A = oracle.csr_to_dense(rp, ci, v, P.N)
        yref = A @ x
        y = P.apply(op, x)
        scale = (np.abs(A) @ np.abs(x)).max()
        assert np.abs(y - yref).max() < 1e-14 * scale
        yr = P.apply_rows(op, x, rows)
        assert np.abs(yr - yref[rows]).max() < 1e-14 * scale
        # the product restricted to the rows' supports gives the same rows
        ye = P.apply_rows_by_elements(op, x, rows)
        assert np.abs(ye - yref[rows]).max() < 1e-14 * scale


def test_support_elements_are_exactly_the_supports():
    """The element set of a row is the box of elements whose span meets
    supp phi_m (p consecutive elements per direction, clipped at the ends),
    checked against the tables' active functions."""
    K, p = (6, 4, 5), 3
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=3)
    P = oracle.Problem(kn, p, ctrl)
    for m in (0, 7, P.N // 3, P.N - 1):
        mi = np.unravel_index(m, P.nfun[::-1])[::-1]
        els = P.support_elements([m])
        want = []
        for e3 in range(K[2]):
            for e2 in range(K[1]):
                for e1 in range(K[0]):
                    e = (e1, e2, e3)
                    if all(e[k] <= mi[k] <= e[k] + p - 1 for k in range(3)):
                        want.append(e1 + K[0] * (e2 + K[1] * e3))
        assert np.array_equal(els, np.array(want))


def test_folded_geometry_is_rejected():
    K, p = (3, 3), 2
    kn, ctrl = inputs.identity_geometry(K, p)
    ctrl = ctrl.copy()
    ctrl[5] = ctrl[10] + 0.3              # fold the map over
    P = oracle.Problem(kn, p, ctrl)
    with pytest.raises(oracle.OracleError):
        P.assemble(oracle.STIFF)


def test_invalid_knots_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.tables_1d(np.array([0, 0, 0.5, 1, 1, 1.0]), 3)     # not open at the left
    with pytest.raises(oracle.OracleError):
        oracle.tables_1d(np.array([0, 0, 0, 0.7, 0.5, 1, 1, 1.0]), 3)


# ------------------------------------------------------------ evaluation (Algorithm 3)

@pytest.mark.parametrize("d,K,p", [(2, (4, 5), 3), (3, (3, 2, 4), 2), (3, (2, 3, 2), 4), (1, (6,), 5)])
def test_eval_reproduces_linear_physical_functions(d, K, p):
    """u_n = gamma . c_n + beta is, by partition of unity and linear
    precision of G = sum c_n phi_n, the function gamma . x + beta of the
    physical point: value gamma . G(xhat) + beta, physical gradient gamma, in
    any (valid) geometry.  A transposed inverse Jacobian or a dropped term
    changes the gradient."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=5)
    P = oracle.Problem(kn, p, ctrl)
    rng = np.random.default_rng(3)
    gam = rng.uniform(-1, 1, d)
    beta = 0.37
    v, g, x = P.eval(ctrl.reshape(-1, d) @ gam + beta)
    assert np.abs(v - (x @ gam + beta)).max() < 1e-13
    assert np.abs(g - gam[None, :]).max() < 1e-12


@pytest.mark.parametrize("K,p", [((3, 2, 4), 3), ((2, 2, 2), 5)])
def test_eval_values_against_scipy_tensor_product(K, p):
    """Values of u = sum u_n phi_n at the Gauss points equal the tensor
    product of scipy B-spline design matrices (an independent evaluation of
    the basis) applied to u; the physical points agree with the same
    contraction of the control points."""
    from scipy.interpolate import BSpline
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=6)
    P = oracle.Problem(kn, p, ctrl)
    u = np.random.default_rng(4).uniform(-1, 1, P.N)
    v, _, x = P.eval(u)
    # 1D design matrices at the Gauss points of every element, points in order
    mats = []
    for k in range(3):
        xs = oracle.tables_1d(kn[k], p)["x"].ravel()
        mats.append(BSpline.design_matrix(xs, kn[k], p - 1).toarray())
    U = u.reshape(P.nfun[2], P.nfun[1], P.nfun[0])        # [i3][i2][i1]
    ref = np.einsum("ai,bj,ck,kji->cba", mats[0], mats[1], mats[2], U).ravel()
    assert np.abs(v - ref).max() < 1e-13
    X = ctrl.reshape(P.nfun[2], P.nfun[1], P.nfun[0], 3)
    refx = np.einsum("ai,bj,ck,kjid->cbad", mats[0], mats[1], mats[2], X).reshape(-1, 3)
    assert np.abs(x - refx).max() < 1e-13
