"""Independent dense brute force for tiny meshes, used only to pin the oracle.

It follows the algebraic form of Sec. 5 (A = Q_Psi^T F Q_Phi) with explicit
dense matrices: 1D values/derivatives from scipy's BSpline (a library
B-spline evaluator, not the oracle's recursion), Gauss points from
numpy's leggauss, the full tensor-product tables by Kronecker products and
the geometry quantities with numpy.linalg.  Shares no code with the oracle.
"""
import numpy as np
from scipy.interpolate import BSpline


def gauss_points_1d(knots, p):
    t = np.asarray(knots, dtype=np.float64)
    br = np.unique(t)
    nodes, weights = np.polynomial.legendre.leggauss(p)
    xs, ws = [], []
    for a, b in zip(br[:-1], br[1:]):
        xs.append(a + (b - a) * (nodes + 1) / 2)
        ws.append(weights * (b - a) / 2)
    return np.concatenate(xs), np.concatenate(ws)


def basis_1d(knots, p, x):
    """Values and derivatives [len(x), n] of all B-splines of order p."""
    t = np.asarray(knots, dtype=np.float64)
    n = len(t) - p
    spl = BSpline(t, np.eye(n), p - 1, extrapolate=False)
    V = spl(x)
    D = spl.derivative()(x) if p > 1 else np.zeros_like(V)
    return np.nan_to_num(V), np.nan_to_num(D)


def dense_bruteforce(knots_list, p, ctrl, coef, op, conv_b=None, diff_A=None):
    """Dense mass (op=1, coefficient 1), stiffness (op=2) or convection
    (op=4: b . grad u tested with v, b = coefficient * conv_b) matrix."""
    d = len(knots_list)
    Xs, Ws, Vs, Ds = [], [], [], []
    for kn in knots_list:
        x, w = gauss_points_1d(kn, p)
        V, D = basis_1d(kn, p, x)
        Xs.append(x); Ws.append(w); Vs.append(V); Ds.append(D)

    def kron_dirs(mats):
        # lexicographic with direction 1 fastest: kron(last, ..., first)
        out = mats[-1]
        for m in mats[-2::-1]:
            out = np.kron(out, m)
        return out

    Qval = kron_dirs(Vs)                       # [Q, N]
    Qder = [kron_dirs([Ds[k] if k == i else Vs[k] for k in range(d)]) for i in range(d)]
    w = kron_dirs([wk[:, None] for wk in Ws])[:, 0]
    ctrl = np.asarray(ctrl).reshape(-1, d)
    G = Qval @ ctrl                            # [Q, d]
    J = np.stack([Qder[k] @ ctrl for k in range(d)], axis=2)   # J[q, i, k] = dG_i/dxhat_k
    det = np.linalg.det(J)
    assert np.all(det > 0)
    Jinv = np.linalg.inv(J)
    kind, val = coef
    if op == 1:
        a = np.ones(len(w))
        F = w * a * np.abs(det)
        return Qval.T @ (F[:, None] * Qval)
    a = np.full(len(w), val) if kind == "const" else 1 + val * np.prod(np.sin(2 * np.pi * G), axis=1)
    if op == 4:
        # physical gradient of phi_n: J^-T grad_hat phi_n; row m carries phi_m
        b = np.asarray(conv_b, dtype=np.float64)[:d]
        A = np.zeros((Qval.shape[1],) * 2)
        for i in range(d):
            # (J^-T g)_i = sum_k Jinv[k, i] g_k
            gi = sum(Jinv[:, k, i][:, None] * Qder[k] for k in range(d))
            A += Qval.T @ ((w * a * np.abs(det) * b[i])[:, None] * gi)
        return A
    Ad = np.eye(d) if diff_A is None else np.asarray(diff_A, dtype=np.float64)
    # K = sum_q (J^-T g_n) . A (J^-T g_m) = g_n . (J^-1 A J^-T) g_m
    C = (w * a * np.abs(det))[:, None, None] * np.einsum("qij,jk,qlk->qil", Jinv, Ad, Jinv)
    A = np.zeros((Qval.shape[1],) * 2)
    for i in range(d):
        for j in range(d):
            A += Qder[i].T @ (C[:, i, j][:, None] * Qder[j])
    return A
