"""Oracle for sum-factorised isogeometric assembly and matrix-free apply.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never imports, links or calls it, and it shares no code with the GPU
path (the seeded input generators are the only common module, and they hold
none of the method's arithmetic).

What it computes (all FP64, plain, unblocked):

* 1D B-spline values and first derivatives at the Gauss points of every
  element, by the literal Cox-de Boor recursion (Example 1 names the
  Cox-de Boor formula for the univariate splines); ``p`` is the *order*
  (degree + 1), as in Sec. 3.2 ("degree nu, order nu+1").
* Gauss-Legendre rule with ``p`` points per element and direction (Example
  "Gauss quadrature" in Sec. 3.2), from ``numpy.polynomial.legendre.leggauss``.
* Element-by-element quadrature sums of the mass, stiffness and convection
  forms (eq. (quadrature:1), pull-back of Example 1) in ``orc.c``; rows are
  test functions, columns trial functions, lexicographic with direction 1
  fastest (Sec. 3.1).  The convection form is the b . grad u term of Example
  1's equation tested with v (derivative on the trial function), with a
  constant vector b scaled by the scalar coefficient.

Readings of the paper adopted here (see the design notes of the repository):
order notation, p Gauss points per element, open knot vectors, the
pull-back |det J| J^-1 A J^-T with J_ik = dG_i/dxhat_k, the coefficient
evaluated at the physical point G(xhat), structural zeros stored.

Mixed-precision bounds: parity unpinned by the paper (it states only that
sum factorisation reproduces the standard matrix up to machine precision);
those modes are checked against this FP64 oracle with measured bounds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")

MASS = 1
STIFF = 2
CONV = 4


def build(force: bool = False) -> str:
    """Compile orc.c with gcc (OpenMP) into liborc.so next to it."""
    src = os.path.join(_HERE, "orc.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


@lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    prob = [ctypes.c_int, i32p, i32p, i32p, i32p, f64p, f64p, f64p, f64p,
            ctypes.c_int, ctypes.c_double]
    lib.orc_pattern.argtypes = prob + [i64p, i64p]
    lib.orc_assemble.argtypes = prob + [ctypes.c_int, i64p, f64p, ctypes.c_int]
    lib.orc_rows.argtypes = prob + [ctypes.c_int, ctypes.c_int64, i64p, ctypes.c_int,
                                    i32p, i64p, f64p, ctypes.c_int]
    lib.orc_apply_rows.argtypes = prob + [ctypes.c_int, f64p, ctypes.c_int64, i64p, f64p,
                                          ctypes.c_int]
    lib.orc_apply.argtypes = prob + [ctypes.c_int, f64p, f64p, ctypes.c_int]
    lib.orc_apply_elements.argtypes = prob + [ctypes.c_int, f64p, ctypes.c_int64, i64p, f64p,
                                              ctypes.c_int]
    lib.orc_eval.argtypes = prob + [f64p, f64p, f64p, f64p, ctypes.c_int]
    lib.orc_measure.argtypes = prob + [f64p]
    lib.orc_set_convection.argtypes = [ctypes.c_double] * 3
    lib.orc_set_convection.restype = None
    lib.orc_set_diffusion.argtypes = [ctypes.POINTER(ctypes.c_double)]
    lib.orc_set_diffusion.restype = None
    for f in (lib.orc_pattern, lib.orc_assemble, lib.orc_rows, lib.orc_apply_rows,
              lib.orc_apply, lib.orc_apply_elements, lib.orc_eval, lib.orc_measure):
        f.restype = ctypes.c_int
    lib.orc_set_defect.argtypes = [ctypes.c_int]
    lib.orc_set_defect.restype = None
    return lib


def set_defect(k: int) -> None:
    """Plant mistake k in the oracle's arithmetic (0 removes it).  Only the
    tests that show the pins catch plausible mistakes use this."""
    _lib().orc_set_defect(int(k))


class OracleError(RuntimeError):
    pass


# ---------------------------------------------------------------- 1D layer

def check_open_knots(knots, p):
    """Open knot vector of order p on [0, 1]: nondecreasing, first and last
    value repeated p times (Corollary on #NZ for open knot vectors)."""
    t = np.asarray(knots, dtype=np.float64)
    if p < 1 or t.ndim != 1 or len(t) < 2 * p:
        raise OracleError("knot vector too short for the order")
    if np.any(np.diff(t) < 0):
        raise OracleError("knots must be nondecreasing")
    if not (np.all(t[:p] == t[0]) and np.all(t[-p:] == t[-1])):
        raise OracleError("knot vector is not open")
    if t[0] != 0.0 or t[-1] != 1.0:
        raise OracleError("knot vector must span [0, 1]")
    inner = t[p:-p]
    for v in np.unique(inner):
        if np.count_nonzero(inner == v) > p:
            raise OracleError("interior knot multiplicity exceeds the order")
    return t


def element_spans(knots, p):
    """Elements = knot spans [t_k, t_{k+1}) of positive length; the B-splines
    active on span k are N_{k-p+1}, ..., N_k."""
    t = np.asarray(knots, dtype=np.float64)
    out = []
    for k in range(p - 1, len(t) - p):
        if t[k + 1] > t[k]:
            out.append((k, t[k], t[k + 1]))
    return out


def cox_de_boor(t, order, i, x, memo=None):
    """N_{i,order}(x) by the Cox-de Boor recursion, 0/0 := 0, half-open
    intervals for order 1."""
    if memo is not None:
        key = (order, i)
        if key in memo:
            return memo[key]
    if order == 1:
        v = 1.0 if t[i] <= x < t[i + 1] else 0.0
    else:
        v = 0.0
        den = t[i + order - 1] - t[i]
        if den != 0.0:
            v += (x - t[i]) / den * cox_de_boor(t, order - 1, i, x, memo)
        den = t[i + order] - t[i + 1]
        if den != 0.0:
            v += (t[i + order] - x) / den * cox_de_boor(t, order - 1, i + 1, x, memo)
    if memo is not None:
        memo[(order, i)] = v
    return v


def cox_de_boor_deriv(t, order, i, x, memo=None):
    """d/dx N_{i,order}(x) = (order-1) [N_{i,order-1}/(t_{i+order-1}-t_i)
    - N_{i+1,order-1}/(t_{i+order}-t_{i+1})], 0/0 := 0."""
    if order == 1:
        return 0.0
    v = 0.0
    den = t[i + order - 1] - t[i]
    if den != 0.0:
        v += (order - 1) / den * cox_de_boor(t, order - 1, i, x, memo)
    den = t[i + order] - t[i + 1]
    if den != 0.0:
        v -= (order - 1) / den * cox_de_boor(t, order - 1, i + 1, x, memo)
    return v


def gauss_legendre(npts):
    return np.polynomial.legendre.leggauss(npts)


def tables_1d(knots, p):
    """Per element: first active function, Gauss points/weights (p per
    element, mapped from [-1, 1]), values and derivatives of the p active
    functions at every point: phi[e, g, j] = N_{first+j}(x_{e,g})."""
    t = check_open_knots(knots, p)
    spans = element_spans(t, p)
    nodes, weights = gauss_legendre(p)
    K = len(spans)
    first = np.zeros(K, dtype=np.int32)
    xq = np.zeros((K, p))
    wq = np.zeros((K, p))
    phi = np.zeros((K, p, p))
    dphi = np.zeros((K, p, p))
    for e, (k, a, b) in enumerate(spans):
        first[e] = k - p + 1
        for g in range(p):
            x = a + (b - a) * (nodes[g] + 1.0) / 2.0
            xq[e, g] = x
            wq[e, g] = weights[g] * (b - a) / 2.0
            memo = {}
            for j in range(p):
                i = k - p + 1 + j
                phi[e, g, j] = cox_de_boor(t, p, i, x, memo)
                dphi[e, g, j] = cox_de_boor_deriv(t, p, i, x, memo)
    nfun = len(t) - p
    return dict(first=first, x=xq, w=wq, phi=phi, dphi=dphi, nfun=nfun, nel=K, p=p)


# ------------------------------------------------------------- problem

COEF_CONST = 0
COEF_SINPROD = 1


class Problem:
    """A single tensor-product patch: knot vectors, order per direction,
    control points [N, d] (lexicographic, direction 1 fastest) and a
    coefficient: ``("const", value)`` or ``("sinprod", alpha)`` meaning
    1 + alpha * prod_i sin(2 pi x_i) at the physical point.  The stiffness
    and convection forms take that coefficient, the mass form c = 1;
    ``conv_b`` is the constant vector b of the convection form and
    ``diff_A`` the constant symmetric matrix A of the stiffness form
    (diffusion a(x) A; default the identity)."""

    def __init__(self, knots, orders, ctrl, coef=("const", 1.0), conv_b=(0.0, 0.0, 0.0), diff_A=None):
        self.d = len(knots)
        self.conv_b = [float(v) for v in conv_b] + [0.0] * (3 - len(conv_b))
        A = np.eye(3)
        if diff_A is not None:
            A[:self.d, :self.d] = np.asarray(diff_A, dtype=np.float64)
        self.diff_A = np.ascontiguousarray(A.ravel())
        if isinstance(orders, int):
            orders = [orders] * self.d
        self.orders = list(orders)
        self.t1d = [tables_1d(k, p) for k, p in zip(knots, self.orders)]
        self.nfun = [t["nfun"] for t in self.t1d]
        self.nel = [t["nel"] for t in self.t1d]
        self.N = int(np.prod(self.nfun))
        self.ctrl = np.ascontiguousarray(ctrl, dtype=np.float64).reshape(self.N, self.d)
        kind, val = coef
        self.coef_kind = {"const": COEF_CONST, "sinprod": COEF_SINPROD}[kind]
        self.coef_val = float(val)
        self._first = np.ascontiguousarray(np.concatenate([t["first"] for t in self.t1d]),
                                           dtype=np.int32)
        self._w = np.ascontiguousarray(np.concatenate([t["w"].ravel() for t in self.t1d]))
        self._phi = np.ascontiguousarray(np.concatenate([t["phi"].ravel() for t in self.t1d]))
        self._dphi = np.ascontiguousarray(np.concatenate([t["dphi"].ravel() for t in self.t1d]))
        self._p = np.asarray(self.orders, dtype=np.int32)
        self._nel = np.asarray(self.nel, dtype=np.int32)
        self._nf = np.asarray(self.nfun, dtype=np.int32)
        self.maxband = int(np.prod([2 * p - 1 for p in self.orders]))

    def _args(self, coef_kind=None, coef_val=None):
        P = ctypes.POINTER
        i32 = P(ctypes.c_int32)
        f64 = P(ctypes.c_double)
        _lib().orc_set_convection(*self.conv_b[:3])
        _lib().orc_set_diffusion(self.diff_A.ctypes.data_as(f64))
        return [self.d, self._p.ctypes.data_as(i32), self._nel.ctypes.data_as(i32),
                self._nf.ctypes.data_as(i32), self._first.ctypes.data_as(i32),
                self._w.ctypes.data_as(f64), self._phi.ctypes.data_as(f64),
                self._dphi.ctypes.data_as(f64), self.ctrl.ctypes.data_as(f64),
                self.coef_kind if coef_kind is None else coef_kind,
                self.coef_val if coef_val is None else coef_val]

    def _coef_for(self, op):
        # mass uses c = 1 (reaction coefficient 1), stiffness the given a(x)
        if op == MASS:
            return COEF_CONST, 1.0
        return self.coef_kind, self.coef_val

    @staticmethod
    def _check(st):
        if st != 0:
            raise OracleError({-1: "invalid input", -3: "det J <= 0", -4: "out of memory"}
                              .get(st, f"status {st}"))

    def pattern(self):
        i64 = ctypes.POINTER(ctypes.c_int64)
        rp = np.zeros(self.N + 1, dtype=np.int64)
        self._check(_lib().orc_pattern(*self._args(), rp.ctypes.data_as(i64), None))
        ci = np.zeros(int(rp[-1]), dtype=np.int64)
        self._check(_lib().orc_pattern(*self._args(), rp.ctypes.data_as(i64),
                                       ci.ctypes.data_as(i64)))
        return rp, ci

    def assemble(self, op, threads=0, pattern=None):
        """Full CSR (row_ptr, col_ind, values) of the mass (op=1), stiffness
        (op=2) or convection (op=4) matrix."""
        rp, ci = pattern if pattern is not None else self.pattern()
        vals = np.zeros(len(ci))
        kind, val = self._coef_for(op)
        self._check(_lib().orc_assemble(*self._args(kind, val), op,
                                        rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        threads))
        return rp, ci, vals

    def rows(self, op, rows, threads=0):
        """Selected rows: list of (cols, vals) with cols ascending."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        n = len(rows)
        cnt = np.zeros(n, dtype=np.int32)
        cols = np.zeros((n, self.maxband), dtype=np.int64)
        vals = np.zeros((n, self.maxband))
        kind, val = self._coef_for(op)
        self._check(_lib().orc_rows(*self._args(kind, val), op, n,
                                    rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    self.maxband,
                                    cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    threads))
        return [(cols[i, :cnt[i]].copy(), vals[i, :cnt[i]].copy()) for i in range(n)]

    def apply(self, op, x, threads=0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.N)
        kind, val = self._coef_for(op)
        f64 = ctypes.POINTER(ctypes.c_double)
        self._check(_lib().orc_apply(*self._args(kind, val), op, x.ctypes.data_as(f64),
                                     y.ctypes.data_as(f64), threads))
        return y

    def apply_rows(self, op, x, rows, threads=0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.zeros(len(rows))
        kind, val = self._coef_for(op)
        f64 = ctypes.POINTER(ctypes.c_double)
        self._check(_lib().orc_apply_rows(*self._args(kind, val), op, x.ctypes.data_as(f64),
                                          len(rows),
                                          rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          y.ctypes.data_as(f64), threads))
        return y

    def support_elements(self, rows):
        """Flattened indices (direction 1 fastest) of the union of the
        elements in supp phi_m over the given rows; element e activates
        functions first[e] .. first[e] + p - 1 (open knots)."""
        rows = np.asarray(rows, dtype=np.int64)
        mi = []
        r = rows.copy()
        for k in range(self.d):
            mi.append(r % self.nfun[k])
            r //= self.nfun[k]
        sel = []
        for k in range(self.d):
            first = self.t1d[k]["first"]
            # element e supports function i iff first[e] <= i <= first[e] + p - 1
            sel.append([np.nonzero((first <= i) & (i <= first + self.orders[k] - 1))[0] for i in mi[k]])
        out = set()
        for j in range(len(rows)):
            axes = [sel[k][j] for k in range(self.d)]
            grid = np.meshgrid(*axes, indexing="ij")
            lin = np.zeros(grid[0].shape, dtype=np.int64)
            stride = 1
            for k in range(self.d):
                lin += grid[k] * stride
                stride *= self.nel[k]
            out.update(lin.ravel().tolist())
        return np.array(sorted(out), dtype=np.int64)

    def apply_rows_by_elements(self, op, x, rows, threads=0):
        """Rows of A x from the element-by-element product over the union of
        the rows' supports (the same sum as ``apply``, restricted to the
        elements those rows need)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        els = np.ascontiguousarray(self.support_elements(rows))
        y = np.zeros(self.N)
        kind, val = self._coef_for(op)
        f64 = ctypes.POINTER(ctypes.c_double)
        self._check(_lib().orc_apply_elements(*self._args(kind, val), op, x.ctypes.data_as(f64),
                                              len(els), els.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              y.ctypes.data_as(f64), threads))
        return y[np.asarray(rows, dtype=np.int64)]

    def nquad(self):
        return int(np.prod([ne * p for ne, p in zip(self.nel, self.orders)]))

    def eval(self, u, threads=0):
        """Values [Q], physical gradients [Q, d] and physical points [Q, d] of
        u = sum u_n phi_n at the quadrature points (lexicographic, direction 1
        fastest), by plain sums over each point's active functions."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        Q = self.nquad()
        val = np.zeros(Q)
        grad = np.zeros((Q, self.d))
        xyz = np.zeros((Q, self.d))
        f64 = ctypes.POINTER(ctypes.c_double)
        self._check(_lib().orc_eval(*self._args(), u.ctypes.data_as(f64), val.ctypes.data_as(f64),
                                    grad.ctypes.data_as(f64), xyz.ctypes.data_as(f64), threads))
        return val, grad, xyz

    def measure(self):
        out = ctypes.c_double(0.0)
        self._check(_lib().orc_measure(*self._args(), ctypes.byref(out)))
        return out.value

    def dense(self, op, threads=0):
        rp, ci, v = self.assemble(op, threads)
        A = np.zeros((self.N, self.N))
        for m in range(self.N):
            A[m, ci[rp[m]:rp[m + 1]]] = v[rp[m]:rp[m + 1]]
        return A


def glue_map(d, nfuns, interfaces):
    """Global numbering of conforming patches glued at faces (Sec. 4,
    Example "Multipatch domains": the functions of two patches that meet on
    an interface are identified, and the glued operator is
    sum_b R_b^T A_b R_b).  nfuns[b][k]: functions of patch b in direction k;
    interfaces: (patch a, face fa, patch b, face fb) with face = 2 k + side
    (side 0 the functions with index 0 in direction k, side 1 the last);
    the remaining directions, in increasing order, are matched index by index.
    Returns (per patch an int64 array of global ids in the patch's
    lexicographic order, the number of global functions).  Plain
    union-find, for the small patches of the tests."""
    offs = [0]
    for nf in nfuns:
        offs.append(offs[-1] + int(np.prod(nf[:d])))
    parent = list(range(offs[-1]))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    def lin(nf, idx):
        m, stride = 0, 1
        for k in range(d):
            m += idx[k] * stride
            stride *= nf[k]
        return m

    for a, fa, b, fb in interfaces:
        ka, sa_, kb, sb_ = fa // 2, fa % 2, fb // 2, fb % 2
        ta = [k for k in range(d) if k != ka]
        tb = [k for k in range(d) if k != kb]
        na, nb = nfuns[a], nfuns[b]
        if [na[k] for k in ta] != [nb[k] for k in tb]:
            raise OracleError("non-conforming interface")
        for t in np.ndindex(*[na[k] for k in ta]):
            ia, ib = [0] * d, [0] * d
            ia[ka] = na[ka] - 1 if sa_ else 0
            ib[kb] = nb[kb] - 1 if sb_ else 0
            for j in range(d - 1):
                ia[ta[j]] = t[j]
                ib[tb[j]] = t[j]
            ra, rb = find(offs[a] + lin(na, ia)), find(offs[b] + lin(nb, ib))
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    gid = {}
    out = []
    for bi in range(len(nfuns)):
        m = np.zeros(offs[bi + 1] - offs[bi], dtype=np.int64)
        for i in range(len(m)):
            r = find(offs[bi] + i)
            if r not in gid:
                gid[r] = len(gid)
            m[i] = gid[r]
        out.append(m)
    return out, len(gid)


def glued_apply(problems, maps, n_global, op, x, threads=0):
    """y = sum_b R_b^T A_b R_b x over glued patches (see glue_map)."""
    y = np.zeros(n_global)
    for P, m in zip(problems, maps):
        np.add.at(y, m, P.apply(op, np.asarray(x)[m], threads))
    return y


def glued_dense(problems, maps, n_global, op, threads=0):
    """The glued matrix sum_b R_b^T A_b R_b, dense."""
    A = np.zeros((n_global, n_global))
    for P, m in zip(problems, maps):
        A[np.ix_(m, m)] += P.dense(op, threads)
    return A


def csr_to_dense(rp, ci, v, n):
    A = np.zeros((n, n))
    for m in range(n):
        A[m, ci[rp[m]:rp[m + 1]]] = v[rp[m]:rp[m + 1]]
    return A
