"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP64 bar (the paper: sum factorization gives the standard matrix up to
machine precision): err_A <= 1e-12 and err_y <= 1e-12, metrics in
tests/gpu_util.py.  FP32 mode: err <= 1e-6, about 16 units of FP32 roundoff
(2^-24): the coefficient tensor is rounded once and each contraction level
sums O(p^2) rounded terms; the largest error measured over every FP32 test,
the 128^3 order-6 patch and the 512-patch set included, is 2.1e-7.
Patterns and row pointers are compared bit-exactly.
"""
import numpy as np
import pytest

import oracle
import paper_1809_05471_amd as sf
from paper_1809_05471_amd import inputs
from tests.gpu_util import GpuPatch, ctx, err_A, err_y, record, sample_rows, straddle_rows

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-6
# BF16 split: operands x = hi + lo in bf16 hold x to 2^-17; a product keeps
# Ahi Bhi + Ahi Blo + Alo Bhi (dropping Alo Blo ~ 2^-18), so each level-2
# term carries about 2^-16 (1.5e-5) relative error before the FP32 and FP64
# sums, which average it down; measured at most 4.2e-6 (orders 2-9)
TOLBF = 2e-5
# FP16 split (matrix-free apply): per element and component C / w = r + s h
# with h in [-1, 1] rounded to FP16, so each coefficient is within
# 2^-12 s w of the FP32 one; s is the half range of C / w over the element
# (the variation of the geometry and the coefficient within it), well below
# max |C / w|.  Measured at most 1.6e-5 over orders 2-9 (err_y).
TOL16 = 1e-4


def _full_parity(knots, p, ctrl, coef, ops=(sf.SF_MASS, sf.SF_STIFF), prec=sf.SF_FP64, tol=TOL64, seed=0,
                 assemble=True, apply=True):
    """Pattern, values and y = A x of the operators against the oracle's full
    assembly (and SpMV) on the same inputs; assemble / apply select what the
    precision mode supports."""
    P = oracle.Problem(knots, p, ctrl, coef)
    x = inputs.random_vector(P.N, seed)
    rp_o, ci_o = P.pattern()
    with GpuPatch(knots, p, ctrl, coef) as g:
        g.prepare(prec=prec)
        rp, ci = g.pattern()
        assert np.array_equal(rp, rp_o)
        assert np.array_equal(ci.astype(np.int64), ci_o)
        out = {}
        for op in ops:
            _, _, v_o = P.assemble(op, pattern=(rp_o, ci_o))
            eA = ey = 0.0
            if assemble:
                v = g.assemble(op, prec)
                assert not np.isnan(v).any()
                eA = err_A(v, v_o)
                record("err_A", prec, eA)
                assert eA <= tol, (op, eA)
            if apply:
                A = oracle.csr_to_dense(rp_o, ci_o, v_o, P.N) if P.N <= 4000 else None
                y_o = P.apply(op, x)
                y = g.apply(op, x, prec)
                absAx = np.abs(A) @ np.abs(x) if A is not None else None
                if absAx is None:
                    absAx = np.zeros(P.N)
                    np.add.at(absAx, np.repeat(np.arange(P.N), np.diff(rp_o)), np.abs(v_o) * np.abs(x[ci_o]))
                ey = err_y(y, y_o, absAx)
                record("err_y", prec, ey)
                assert ey <= tol, (op, ey)
            out[op] = (eA, ey)
        return out


def test_small_2d_identity_16x16_p3():
    """d = 2, 16 x 16 elements, order 3, identity geometry, a = c = 1."""
    w = inputs.workload_small_2d()
    _full_parity(w["knots"], w["p"], w["ctrl"], w["coef"])


@pytest.mark.parametrize("K,p", [((9, 19, 21), 2), ((6, 15, 17), 3), ((4, 9, 17), 4), ((2, 6, 17), 5),
                                 ((1, 5, 17), 6), ((60, 5, 7), 2), ((45, 4, 9), 3), ((25, 4, 9), 4),
                                 ((14, 3, 6), 5), ((9, 2, 7), 6)])
def test_3d_full_parity_several_tiles(K, p):
    """Several direction-1 row tiles of the level-1/2 kernel and several
    direction-3 row segments of the level-3 kernel (ragged last ones), apply
    tiles with ragged edges, perturbed geometry, variable coefficient."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=1)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5))


def _random_shapes(n, seed, budget=1.2e9):
    """Seeded random ragged 3D shapes: 1..10 elements per direction, orders
    2..7, with the oracle's cost (elements x p^9) under `budget`."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        p = int(rng.integers(2, 8))
        K = tuple(int(k) for k in rng.integers(1, 11, size=3))
        if np.prod(K) * float(p) ** 9 <= budget:
            out.append((K, p))
    return out


@pytest.mark.parametrize("K,p", _random_shapes(10, seed=2024))
def test_3d_random_shapes(K, p):
    """Random ragged shapes: single elements, fewer elements than p, row
    tiles and level-2 windows cut at the mesh edges in every combination the
    draw produces; full matrices and products against the oracle."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=7)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5))


@pytest.mark.parametrize("K,p", _random_shapes(6, seed=77))
def test_3d_random_shapes_fp32(K, p):
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=8)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_FP32, tol=TOL32)


@pytest.mark.parametrize("K,p", [((7, 3, 5), 2), ((3, 4, 3), 4), ((2, 3, 2), 6)])
def test_3d_fp32_mode(K, p):
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=4)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_FP32, tol=TOL32)


@pytest.mark.parametrize("K,p", [((7, 3, 5), 2), ((13, 4, 6), 3), ((21, 3, 5), 4), ((3, 4, 3), 5), ((2, 3, 2), 6),
                                 ((2, 3, 2), 7), ((2, 2, 2), 8), ((1, 1, 2), 9)])
def test_3d_bf16_split_mode(K, p):
    """Level 2 of the assembly on bf16 matrix cores with hi/lo split operands
    and FP32 accumulation (FP32 coefficients and level 1, FP64 level 3 and
    values); the apply runs its FP32 path.  Parity unpinned by the paper:
    checked against the FP64 oracle with the bound TOLBF.  BF16 split is a
    mode of the assembly: the apply refuses it."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=4)
    res = _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_BF16_SPLIT, tol=TOLBF, apply=False)
    # the split keeps far more than bf16 alone (2^-9 ~ 2e-3) would
    assert max(eA for eA, _ in res.values()) < 1e-4


@pytest.mark.parametrize("K,p", [((7, 3, 5), 2), ((13, 4, 6), 3), ((21, 3, 5), 4), ((3, 4, 3), 5), ((4, 3, 2), 6),
                                 ((2, 3, 2), 7), ((2, 2, 2), 8), ((1, 1, 2), 9)])
def test_3d_fp16_split_apply(K, p):
    """Matrix-free apply with the coefficients stored as FP16 residuals of a
    per-element FP32 reference and scale (2 bytes per component), several
    tiles and ragged edges, mass and stiffness, against the FP64 oracle with
    the bound TOL16; the assembly refuses the mode."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=14)
    res = _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_FP16_SPLIT, tol=TOL16, assemble=False)
    # far more than FP16 alone would keep (2^-11 ~ 5e-4 of the values)
    assert max(ey for _, ey in res.values()) < 5e-5


@pytest.mark.parametrize("K,p", [((2, 3, 2), 7), ((2, 2, 2), 8), ((1, 1, 2), 9)])
def test_3d_fp32_high_order(K, p):
    """FP32 contractions at orders 7-9, where the level-1/2 tiles are 3, 2
    and 3 rows m1 high: several tiles per plane and a ragged last one."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=5)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_FP32, tol=TOL32)


@pytest.mark.parametrize("K,p", [((17,), 2), ((5,), 5), ((30,), 9)])
def test_1d(K, p):
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=2)
    _full_parity(kn, p, ctrl, ("sinprod", 0.3))


@pytest.mark.parametrize("K,p", [((7, 5), 2), ((3, 4), 6), ((2, 3), 9)])
def test_2d_perturbed(K, p):
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=6)
    _full_parity(kn, p, ctrl, ("sinprod", 0.7))


@pytest.mark.parametrize("K,p", [((2, 3, 2), 7), ((1, 2, 2), 8), ((1, 1, 2), 9)])
def test_3d_high_order(K, p):
    """Orders 7-9: geometry step, assembly and apply."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=3)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5))


@pytest.mark.parametrize("K,p,mb", [((6, 7, 13), 3, 1), ((3, 4, 11), 5, 1), ((30, 20, 9), 2, 1)])
def test_3d_assembly_in_chunks(monkeypatch, K, p, mb):
    """A workspace cap far below the patch's level-2 partials forces chunks of
    element layers in direction 3 (down to the minimum of p - 1 layers);
    entries that straddle two chunks are summed across them."""
    monkeypatch.setenv("SFIGA_WORKSPACE_MB", str(mb))
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=12)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5))
    _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_FP32, tol=TOL32)


def test_mass_and_stiffness_share_pattern_and_assembly_is_deterministic():
    kn, ctrl = inputs.perturbed_geometry((5, 6, 7), 3, seed=8)
    with GpuPatch(kn, 3, ctrl, ("sinprod", 0.5)) as g:
        g.prepare()
        a = g.assemble(sf.SF_STIFF)
        b = g.assemble(sf.SF_STIFF)
        assert np.array_equal(a.view(np.int64), b.view(np.int64))


def test_qp_values_coefficient_matches_builtin():
    """SF_COEF_QPVALUES fed with a(G(x)) evaluated at sf_patch_quad_points
    reproduces SF_COEF_SINPROD."""
    import torch
    kn, ctrl = inputs.perturbed_geometry((4, 5, 3), 3, seed=9)
    with GpuPatch(kn, 3, ctrl, ("sinprod", 0.5)) as g:
        g.prepare(sf.SF_STIFF)
        ref = g.assemble(sf.SF_STIFF)
        xyz = torch.empty((g.Q, 3), dtype=torch.float64, device="cuda")
        sf.sf_patch_quad_points(ctx(), g.h, xyz)
        a = 1.0 + 0.5 * torch.prod(torch.sin(2 * np.pi * xyz), dim=1)
        a = a.contiguous()
        sf.sf_patch_set_coef(ctx(), g.h, sf.SF_STIFF, sf.SF_COEF_QPVALUES, qp_values=a)
        g.prepare(sf.SF_STIFF)
        v = g.assemble(sf.SF_STIFF)
        assert err_A(v, ref) <= 1e-14
        # quadrature points agree with the oracle's geometry map
        P = oracle.Problem(kn, 3, ctrl)
        assert abs(P.measure() - 1.0) < 0.1


def _abs_ax_scale(P, op, x, rows, nscale=4):
    """Scale of err_y: max over up to nscale interior rows of sum_n |A_mn| |x_n|
    (rows with full bands, where that sum is largest), from the oracle's row
    assembly."""
    idx = np.stack(np.unravel_index(rows, P.nfun[::-1])[::-1], axis=1)
    p = max(P.orders)
    inner = [r for r, m in zip(rows, idx) if all(p - 1 <= m[k] <= P.nfun[k] - p for k in range(P.d))]
    pick = (inner or list(rows))[:nscale]
    return max(np.abs(v) @ np.abs(x[c]) for c, v in P.rows(op, pick))


def _sampled_parity(w, ops, prec=sf.SF_FP64, tol=TOL64, nrandom=48, assemble=True, coarse=False, band="grid"):
    """Sampled rows of the assembled matrix (against the oracle's row
    assembly) and of y = A x (against the oracle's element-by-element product
    over the rows' supports), including the rows whose bands are clipped by
    the boundary in each direction."""
    kn, p, ctrl, coef, x = w["knots"], w["p"], w["ctrl"], w["coef"], w["x"]
    P = oracle.Problem(kn, p, ctrl, coef)
    rows = sample_rows(P.nfun, np.random.default_rng(5), nrandom, coarse, p=p, band=band)
    res = {}
    with GpuPatch(kn, p, ctrl, coef) as g:
        g.prepare(prec=prec)
        if assemble:
            rp, ci = g.pattern()
            assert rp[-1] == g.nnz
        for op in ops:
            if assemble:
                ref = P.rows(op, rows)
                vmax = max(np.abs(v).max() for _, v in ref)
                vals = g.assemble(op, prec)
                worst = 0.0
                for r, (c, v) in zip(rows, ref):
                    cg = ci[rp[r]:rp[r + 1]]
                    assert np.array_equal(cg.astype(np.int64), c)
                    worst = max(worst, float(np.abs(vals[rp[r]:rp[r + 1]] - v).max()))
                record("err_A", prec, worst / vmax)
                assert worst / vmax <= tol, (op, worst / vmax)
                res[("A", op)] = worst / vmax
            y = g.apply(op, x, prec)
            y_o = P.apply_rows_by_elements(op, x, rows)
            ey = float(np.abs(y[rows] - y_o).max() / _abs_ax_scale(P, op, x, rows))
            record("err_y", prec, ey)
            assert ey <= tol, (op, ey)
            res[("y", op)] = ey
    return res


def test_3d_48cubed_p4_sampled_rows():
    """Full-size d = 3, 48^3 elements, order 4, perturbed geometry,
    a = 1 + 0.5 sin sin sin: sampled rows of K (and M) and of y = A x, in the
    launch configuration the benchmark times."""
    w = inputs.workload_3d((48, 48, 48), 4)
    _sampled_parity(w, (sf.SF_STIFF, sf.SF_MASS))


def test_3d_48cubed_p4_pattern_and_invariants():
    """Bit-exact pattern against the oracle's, symmetry and K 1 = 0 on the
    full matrix."""
    import scipy.sparse as sp
    w = inputs.workload_3d((48, 48, 48), 4)
    P = oracle.Problem(w["knots"], 4, w["ctrl"], w["coef"])
    rp_o, ci_o = P.pattern()
    with GpuPatch(w["knots"], 4, w["ctrl"], w["coef"]) as g:
        g.prepare(sf.SF_STIFF)
        rp, ci = g.pattern()
        assert np.array_equal(rp, rp_o)
        assert np.array_equal(ci.astype(np.int64), ci_o)
        v = g.assemble(sf.SF_STIFF)
        A = sp.csr_matrix((v, ci, rp), shape=(g.N, g.N))
        scale = np.abs(v).max()
        assert abs(A - A.T).max() <= 1e-13 * scale
        y = A @ np.ones(g.N)
        assert np.abs(y).max() <= 1e-12 * scale
        y1 = g.apply(sf.SF_STIFF, np.ones(g.N))
        assert np.abs(y1).max() <= 1e-12 * scale


_LARGE = {}


def _large_reference():
    """Oracle rows of the 128^3 order-6 patch, computed once for both
    precisions: corner, edge, face and interior rows with the clipped-band
    indices 1, p-2, N-p+1, N-2 in every direction, rows whose m3 lies within
    p-1 layers after every level-3 chunk boundary of the FP64 and of the FP32
    workspace (entries summed across two chunks), and random rows."""
    if not _LARGE:
        w = inputs.workload_3d((128, 128, 128), 6)
        P = oracle.Problem(w["knots"], 6, w["ctrl"], w["coef"])
        n = P.nfun[0]
        picks12 = [(0, 0), (n // 2, n // 2), (n - 1, 1), (4, n - 5)]
        extra = straddle_rows(P.nfun, P.nel, 6, 8, picks12) + straddle_rows(P.nfun, P.nel, 6, 4, picks12)
        rows = sample_rows(P.nfun, np.random.default_rng(11), 12, coarse=True, p=6, extra=extra)
        ref = P.rows(sf.SF_STIFF, rows)
        _LARGE.update(w=w, P=P, rows=rows, ref=ref,
                      y=P.apply_rows_by_elements(sf.SF_STIFF, w["x"], rows),
                      scale=_abs_ax_scale(P, sf.SF_STIFF, w["x"], rows))
    return _LARGE


@pytest.mark.parametrize("prec,tol", [(sf.SF_FP64, TOL64), (sf.SF_FP32, TOL32)])
def test_3d_128cubed_p6_sampled_rows(monkeypatch, prec, tol):
    """Large patch: d = 3, 128^3 elements, order 6 (N = 2,352,637, nnz =
    2,942,649,737), perturbed geometry, a = 1 + 0.5 sin sin sin; stiffness
    assembly and y = A x, compared with the oracle on about 500 sampled rows
    (clipped bands, chunk boundaries); only those rows leave the device.
    The workspace is capped at 4 GiB here, so the assembly runs in 7 chunks
    of element layers in FP64 and 4 in FP32 (by default the whole patch fits
    one chunk, as every smaller test's does)."""
    import torch
    monkeypatch.setenv("SFIGA_WORKSPACE_MB", "4096")
    L = _large_reference()
    w, P, rows, ref = L["w"], L["P"], L["rows"], L["ref"]
    kn, p, ctrl, coef, x = w["knots"], w["p"], w["ctrl"], w["coef"], w["x"]
    assert len(rows) > 400
    vmax = max(np.abs(v).max() for _, v in ref)
    with GpuPatch(kn, p, ctrl, coef) as g:
        assert (g.N, g.nnz) == (2352637, 2942649737)
        g.prepare(sf.SF_STIFF, prec)
        rp = torch.empty(g.N + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(g.nnz, dtype=torch.int32, device="cuda")
        sf.sf_csr_pattern(ctx(), g.h, rp, ci)
        v = torch.empty(g.nnz, dtype=torch.float64, device="cuda")
        sf.sf_assemble(ctx(), g.h, sf.SF_STIFF, prec, val_stiff=v)
        torch.cuda.synchronize()
        rpn = rp.cpu().numpy()
        assert rpn[-1] == g.nnz
        # gather the sampled rows on the device, then copy once
        seg = [np.arange(rpn[r], rpn[r + 1]) for r in rows]
        gidx = torch.as_tensor(np.concatenate(seg)).cuda()
        vg, cg = v[gidx].cpu().numpy(), ci[gidx].cpu().numpy()
        worst, o = 0.0, 0
        for (c, vr), sg in zip(ref, seg):
            assert np.array_equal(cg[o:o + len(sg)].astype(np.int64), c)
            worst = max(worst, float(np.abs(vg[o:o + len(sg)] - vr).max()))
            o += len(sg)
        record("err_A", prec, worst / vmax)
        assert worst / vmax <= tol, worst / vmax
        del v, ci, gidx
        y = g.apply(sf.SF_STIFF, x, prec)
        ey = float(np.abs(y[rows] - L["y"]).max() / L["scale"])
        record("err_y", prec, ey)
        assert ey <= tol, ey
        # K 1 = 0 on every row (partition of unity), through the matrix-free path
        y1 = g.apply(sf.SF_STIFF, np.ones(g.N), prec)
        assert np.abs(y1).max() <= (1e-12 if prec == sf.SF_FP64 else 1e-5) * vmax


def test_3d_128cubed_p6_fp16_split_apply():
    """The 128^3 order-6 patch: matrix-free apply with the FP16-split
    coefficient storage, on the sampled rows of the large-patch reference."""
    L = _large_reference()
    w = L["w"]
    with GpuPatch(w["knots"], w["p"], w["ctrl"], w["coef"]) as g:
        g.prepare(sf.SF_STIFF, sf.SF_FP16_SPLIT)
        y = g.apply(sf.SF_STIFF, w["x"], sf.SF_FP16_SPLIT)
        ey = float(np.abs(y[L["rows"]] - L["y"]).max() / L["scale"])
        record("err_y", sf.SF_FP16_SPLIT, ey)
        assert ey <= TOL16, ey


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8, 9])
def test_order_sweep_apply_sampled(p):
    """d = 3, K = 127 - p per direction (N = 126^3 for every order), matrix-free
    stiffness apply on sampled rows (clipped-band indices in every direction:
    every combination up to order 7, one direction at a time above), FP64 and
    FP32."""
    w = inputs.workload_order_sweep(p)
    coarse = p >= 6
    band = "grid" if p <= 7 else "cross"
    _sampled_parity(w, (sf.SF_STIFF,), nrandom=4 if coarse else 16, assemble=False, coarse=coarse, band=band)
    if p in (2, 4, 6, 8):
        _sampled_parity(w, (sf.SF_STIFF,), prec=sf.SF_FP32, tol=TOL32, nrandom=4, assemble=False, coarse=True,
                        band="cross")
    if p in (3, 5, 7, 9):
        _sampled_parity(w, (sf.SF_STIFF,), prec=sf.SF_FP16_SPLIT, tol=TOL16, nrandom=4, assemble=False, coarse=True,
                        band="cross")


@pytest.mark.parametrize("npatch,kmax,pmax,side", [(6, 6, 6, False), (6, 6, 6, True), (30, 8, 4, True)])
def test_batched_patches(npatch, kmax, pmax, side):
    """Independent patches of different sizes and orders in one batch:
    persistent kernels per order with autotuned tiles; on a side stream every
    call is one captured HIP graph, replayed.  Block-diagonal CSR and y
    against the oracle patch by patch, on every replay."""
    import torch
    from tests.gpu_util import side_ctx
    c, stream = side_ctx() if side else (ctx(), torch.cuda.current_stream())
    Ks, ps = inputs.batched_draw(npatch, seed=2, kmin=2, kmax=kmax, pmin=2, pmax=pmax)
    patches, probs, xs = [], [], []
    with torch.cuda.stream(stream):
        for b in range(npatch):
            kn, ctrl, x = inputs.batched_patch(b, Ks[b], ps[b])
            g = GpuPatch(kn, int(ps[b]), ctrl, context=c)
            g.prepare()
            patches.append(g)
            probs.append(oracle.Problem(kn, int(ps[b]), ctrl))
            xs.append(x)
        ref = []
        for b, P in enumerate(probs):
            rp_o, ci_o = P.pattern()
            vals = {op: P.assemble(op, pattern=(rp_o, ci_o))[2] for op in (sf.SF_MASS, sf.SF_STIFF)}
            A = oracle.csr_to_dense(rp_o, ci_o, vals[sf.SF_STIFF], P.N)
            ref.append((rp_o, ci_o, vals, A @ xs[b], np.abs(A) @ np.abs(xs[b])))
        try:
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            ro, zo = sf.sf_batch_offsets(c, bt, npatch)
            Ntot, Z = int(ro[-1]), int(zo[-1])
            rp = torch.empty(Ntot + 1, dtype=torch.int64, device="cuda")
            ci = torch.empty(Z, dtype=torch.int32, device="cuda")
            vm = torch.empty(Z, dtype=torch.float64, device="cuda")
            vs = torch.empty(Z, dtype=torch.float64, device="cuda")
            xall = torch.as_tensor(np.concatenate(xs)).cuda()
            y = torch.empty(Ntot, dtype=torch.float64, device="cuda")
            for rep in range(3):             # first call tunes and captures; then replays
                vm.fill_(float("nan"))
                vs.fill_(float("nan"))
                y.fill_(float("nan"))
                sf.sf_batch_assemble(c, bt, sf.SF_MASS | sf.SF_STIFF, sf.SF_FP64, rp, ci, vm, vs)
                sf.sf_batch_apply(c, bt, sf.SF_STIFF, sf.SF_FP64, xall, y)
                stream.synchronize()
                rpn, cin, vmn, vsn, yn = (t.cpu().numpy() for t in (rp, ci, vm, vs, y))
                for b in range(npatch):
                    rp_o, ci_o, vals, y_o, absAx = ref[b]
                    r0, r1, z0, z1 = ro[b], ro[b + 1], zo[b], zo[b + 1]
                    assert np.array_equal(rpn[r0:r1 + 1] - z0, rp_o), (rep, b)
                    assert np.array_equal(cin[z0:z1].astype(np.int64) - r0, ci_o), (rep, b)
                    assert err_A(vmn[z0:z1], vals[sf.SF_MASS]) <= TOL64, (rep, b)
                    assert err_A(vsn[z0:z1], vals[sf.SF_STIFF]) <= TOL64, (rep, b)
                    assert err_y(yn[r0:r1], y_o, absAx) <= TOL64, (rep, b)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()


_B512 = {}


def _batch512_reference():
    """Oracle rows of the 512-patch workload (K ~ U{4..32} per direction,
    p ~ U{2..6}, seed 2), computed once for both precisions.  Per patch:
    the first and last row, the centre row and a row with clipped bands in
    every direction, plus two random rows for orders up to 5 (the oracle's
    row cost grows as p^9); stiffness rows for all of them, mass rows for the
    first two.  y = K x on the same rows from the assembled oracle rows."""
    if not _B512:
        Ks, ps = inputs.batched_draw(512, seed=2)
        pats = []
        for b in range(512):
            p = int(ps[b])
            kn, ctrl, x = inputs.batched_patch(b, Ks[b], p)
            P = oracle.Problem(kn, p, ctrl)
            n = P.nfun
            rng = np.random.default_rng([3, b])
            rows = [0, P.N - 1, int(np.ravel_multi_index([v // 2 for v in n][::-1], n[::-1])),
                    int(np.ravel_multi_index([min(p - 2, n[2] - 1), n[1] - 2, 1], n[::-1]))]
            if p <= 5:
                rows += [int(v) for v in rng.integers(0, P.N, 2)]
            rows = np.array(sorted(set(rows)), dtype=np.int64)
            ks = P.rows(sf.SF_STIFF, rows)
            km = P.rows(sf.SF_MASS, rows[:2])
            if b % 64 == 63:
                print(f"  oracle rows of patch {b + 1}/512", flush=True)
            pats.append(dict(kn=kn, ctrl=ctrl, p=p, x=x, rows=rows, ks=ks, km=km,
                             y=np.array([v @ x[c] for c, v in ks]),
                             absAx=max(np.abs(v) @ np.abs(x[c]) for c, v in ks)))
        _B512["pats"] = pats
    return _B512["pats"]


@pytest.mark.parametrize("prec,tol", [(sf.SF_FP64, TOL64), (sf.SF_FP32, TOL32)])
def test_batched_512_patches_full_size(prec, tol):
    """The batched workload at its stated size: 512 independent patches,
    K ~ U{4..32} per direction (every order 2..6 has patches with 32 elements
    in some direction), p ~ U{2..6}, perturbed geometries, mass + stiffness
    CSR assembly and y = K x through the persistent kernels, captured into HIP
    graphs on a side stream; the first call tunes and captures, the second
    replays.  Sampled rows of every patch (pattern bit-exact, values, y)
    against the oracle after each call."""
    import torch
    from tests.gpu_util import side_ctx
    pats = _batch512_reference()
    c, stream = side_ctx()
    with torch.cuda.stream(stream):
        patches = []
        try:
            for q in pats:
                g = GpuPatch(q["kn"], q["p"], q["ctrl"], context=c)
                patches.append(g)
                g.prepare(prec=prec)
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            ro, zo = sf.sf_batch_offsets(c, bt, len(pats))
            Ntot, Z = int(ro[-1]), int(zo[-1])
            assert Z == 2120728236
            rp = torch.empty(Ntot + 1, dtype=torch.int64, device="cuda")
            ci = torch.empty(Z, dtype=torch.int32, device="cuda")
            vm = torch.empty(Z, dtype=torch.float64, device="cuda")
            vs = torch.empty(Z, dtype=torch.float64, device="cuda")
            xall = torch.as_tensor(np.concatenate([q["x"] for q in pats])).cuda()
            y = torch.empty(Ntot, dtype=torch.float64, device="cuda")
            for rep in range(2):
                vm.fill_(float("nan"))
                vs.fill_(float("nan"))
                y.fill_(float("nan"))
                sf.sf_batch_assemble(c, bt, sf.SF_MASS | sf.SF_STIFF, prec, rp, ci, vm, vs)
                sf.sf_batch_apply(c, bt, sf.SF_STIFF, prec, xall, y)
                stream.synchronize()
                rpn, yn = rp.cpu().numpy(), y.cpu().numpy()
                assert rpn[-1] == Z
                segs = []
                for b, q in enumerate(pats):
                    for r in q["rows"]:
                        a0, a1 = rpn[ro[b] + r], rpn[ro[b] + r + 1]
                        segs.append(np.arange(a0, a1))
                gidx = torch.as_tensor(np.concatenate(segs)).cuda()
                cin, vmn, vsn = (t[gidx].cpu().numpy() for t in (ci, vm, vs))
                del gidx
                o, k = 0, 0
                worst_a, worst_y = 0.0, 0.0
                for b, q in enumerate(pats):
                    vmax = max(np.abs(v).max() for _, v in q["ks"])
                    mmax = max(np.abs(v).max() for _, v in q["km"])
                    for j, r in enumerate(q["rows"]):
                        n = len(segs[k])
                        cols, vref = q["ks"][j]
                        assert np.array_equal(cin[o:o + n].astype(np.int64) - ro[b], cols), (rep, b, r)
                        worst_a = max(worst_a, float(np.abs(vsn[o:o + n] - vref).max()) / vmax)
                        if j < len(q["km"]):
                            worst_a = max(worst_a, float(np.abs(vmn[o:o + n] - q["km"][j][1]).max()) / mmax)
                        o += n
                        k += 1
                    worst_y = max(worst_y, float(np.abs(yn[ro[b] + q["rows"]] - q["y"]).max()) / q["absAx"])
                record("err_A", prec, worst_a)
                record("err_y", prec, worst_y)
                print(f"  call {rep}: err_A {worst_a:.2e} err_y {worst_y:.2e}", flush=True)
                assert worst_a <= tol, (rep, worst_a)
                assert worst_y <= tol, (rep, worst_y)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()
            torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tol", [(sf.SF_FP32, TOL32), (sf.SF_BF16_SPLIT, TOLBF)])
def test_batched_mixed_precision(prec, tol):
    """The batched path in the reduced-precision modes (the 512-patch workload
    runs FP32 contractions), on a side stream with graph replay."""
    import torch
    from tests.gpu_util import side_ctx
    c, stream = side_ctx()
    Ks, ps = inputs.batched_draw(12, seed=5, kmin=2, kmax=6, pmin=2, pmax=5)
    with torch.cuda.stream(stream):
        patches, refs = [], []
        for b in range(12):
            kn, ctrl, x = inputs.batched_patch(b, Ks[b], ps[b])
            g = GpuPatch(kn, int(ps[b]), ctrl, context=c)
            g.prepare(prec=prec)
            patches.append(g)
            P = oracle.Problem(kn, int(ps[b]), ctrl)
            rp_o, ci_o = P.pattern()
            refs.append({op: P.assemble(op, pattern=(rp_o, ci_o))[2] for op in (sf.SF_MASS, sf.SF_STIFF)})
        try:
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            ro, zo = sf.sf_batch_offsets(c, bt, 12)
            Z = int(zo[-1])
            rp = torch.empty(int(ro[-1]) + 1, dtype=torch.int64, device="cuda")
            ci = torch.empty(Z, dtype=torch.int32, device="cuda")
            vm = torch.empty(Z, dtype=torch.float64, device="cuda")
            vs = torch.empty(Z, dtype=torch.float64, device="cuda")
            for rep in range(2):
                vs.fill_(float("nan"))
                sf.sf_batch_assemble(c, bt, sf.SF_MASS | sf.SF_STIFF, prec, rp, ci, vm, vs)
                stream.synchronize()
                vmn, vsn = vm.cpu().numpy(), vs.cpu().numpy()
                for b in range(12):
                    z0, z1 = zo[b], zo[b + 1]
                    assert err_A(vmn[z0:z1], refs[b][sf.SF_MASS]) <= tol, (rep, b)
                    assert err_A(vsn[z0:z1], refs[b][sf.SF_STIFF]) <= tol, (rep, b)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()


def test_batched_fp16_split_apply():
    """Batched matrix-free apply with the FP16-split coefficient storage
    (persistent kernels, captured graph on a side stream, replayed), patch by
    patch against the oracle's product."""
    import torch
    from tests.gpu_util import side_ctx
    c, stream = side_ctx()
    Ks, ps = inputs.batched_draw(12, seed=6, kmin=2, kmax=7, pmin=2, pmax=6)
    with torch.cuda.stream(stream):
        patches, refs, xs = [], [], []
        for b in range(12):
            kn, ctrl, x = inputs.batched_patch(b, Ks[b], ps[b])
            g = GpuPatch(kn, int(ps[b]), ctrl, context=c)
            g.prepare(sf.SF_STIFF, sf.SF_FP16_SPLIT)
            patches.append(g)
            P = oracle.Problem(kn, int(ps[b]), ctrl)
            rp_o, ci_o, v_o = P.assemble(sf.SF_STIFF)
            A = oracle.csr_to_dense(rp_o, ci_o, v_o, P.N)
            refs.append((A @ x, np.abs(A) @ np.abs(x)))
            xs.append(x)
        try:
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            ro, _ = sf.sf_batch_offsets(c, bt, 12)
            xall = torch.as_tensor(np.concatenate(xs)).cuda()
            y = torch.empty(int(ro[-1]), dtype=torch.float64, device="cuda")
            for rep in range(3):
                y.fill_(float("nan"))
                sf.sf_batch_apply(c, bt, sf.SF_STIFF, sf.SF_FP16_SPLIT, xall, y)
                stream.synchronize()
                yn = y.cpu().numpy()
                for b in range(12):
                    ey = err_y(yn[ro[b]:ro[b + 1]], *refs[b])
                    record("err_y", sf.SF_FP16_SPLIT, ey)
                    assert ey <= TOL16, (rep, b, ey)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()


def test_batched_equals_single_patch():
    """Tile shapes (tuned separately for the single-patch and the batched
    launches) do not change the summation order of any entry: the batched
    FP64 assembly equals the single-patch one to the last bits (the two
    launches are separate compilations of the same block code, so only
    contraction of multiply-adds may differ)."""
    import torch
    from tests.gpu_util import side_ctx
    c, stream = side_ctx()
    Ks, ps = inputs.batched_draw(8, seed=9, kmin=3, kmax=9, pmin=2, pmax=5)
    with torch.cuda.stream(stream):
        patches = []
        for b in range(8):
            kn, ctrl, _ = inputs.batched_patch(b, Ks[b], ps[b])
            g = GpuPatch(kn, int(ps[b]), ctrl, coef=("sinprod", 0.5), context=c)
            g.prepare(sf.SF_STIFF)
            patches.append(g)
        try:
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            ro, zo = sf.sf_batch_offsets(c, bt, 8)
            Z = int(zo[-1])
            rp = torch.empty(int(ro[-1]) + 1, dtype=torch.int64, device="cuda")
            ci = torch.empty(Z, dtype=torch.int32, device="cuda")
            vs = torch.empty(Z, dtype=torch.float64, device="cuda")
            sf.sf_batch_assemble(c, bt, sf.SF_STIFF, sf.SF_FP64, rp, ci, None, vs)
            stream.synchronize()
            vsn = vs.cpu().numpy()
            for b, g in enumerate(patches):
                v = torch.empty(g.nnz, dtype=torch.float64, device="cuda")
                sf.sf_assemble(c, g.h, sf.SF_STIFF, sf.SF_FP64, val_stiff=v)
                stream.synchronize()
                assert err_A(vsn[zo[b]:zo[b + 1]], v.cpu().numpy()) <= 4e-16, b
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()


def test_async_prepare_and_geometry_check():
    """sf_patch_prepare_async queues the same geometry kernel as
    sf_patch_prepare: the stiffness assembled after it is bitwise the same.
    A folded map's det J failure is not returned by the call but by
    sf_patch_geometry_check, which clears it (the next check passes)."""
    import torch
    w = inputs.workload_3d((6, 5, 7), 3)
    with GpuPatch(w["knots"], 3, w["ctrl"], coef=("sinprod", 0.5)) as g:
        g.prepare(sf.SF_STIFF)
        a_sync = g.assemble(sf.SF_STIFF)
        sf.sf_patch_prepare_async(g.ctx, g.h, sf.SF_STIFF, sf.SF_FP64)
        a_async = g.assemble(sf.SF_STIFF)
        sf.sf_patch_geometry_check(g.ctx, g.h)
        assert np.array_equal(a_sync.view(np.int64), a_async.view(np.int64))
    kn, ctrl = inputs.identity_geometry((3, 3, 3), 3)
    folded = ctrl.copy()
    folded[:, 0] = -folded[:, 0]                    # mirrored map: det J < 0 everywhere
    with GpuPatch(kn, 3, folded) as g:
        sf.sf_patch_prepare_async(g.ctx, g.h, sf.SF_STIFF, sf.SF_FP64)   # no error here
        with pytest.raises(sf.SfError) as e:
            sf.sf_patch_geometry_check(g.ctx, g.h)
        assert e.value.status == sf.SF_EGEOM
        sf.sf_patch_geometry_check(g.ctx, g.h)       # cleared by the check
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,tol", [(sf.SF_FP64, TOL64), (sf.SF_FP32, TOL32)])
def test_apply_follows_a_new_coefficient(prec, tol):
    """Order 6 (tiled coefficient copy of the apply in FP64, the coef_index
    layout in FP32): apply, change the stiffness coefficient, prepare again,
    apply again; both products against the oracle (ragged apply tiles in
    directions 1 and 2, several layers)."""
    K, p = (7, 8, 5), 6
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=23)
    x = None
    with GpuPatch(kn, p, ctrl, ("sinprod", 0.5)) as g:
        for alpha in (0.5, -0.7):
            P = oracle.Problem(kn, p, ctrl, ("sinprod", alpha))
            if x is None:
                x = inputs.random_vector(P.N, 5)
            sf.sf_patch_set_coef(g.ctx, g.h, sf.SF_STIFF, sf.SF_COEF_SINPROD, alpha)
            g.prepare(sf.SF_MASS | sf.SF_STIFF, prec)
            for op in (sf.SF_STIFF, sf.SF_MASS):
                rp_o, ci_o, v_o = P.assemble(op)
                absAx = np.zeros(P.N)
                np.add.at(absAx, np.repeat(np.arange(P.N), np.diff(rp_o)), np.abs(v_o) * np.abs(x[ci_o]))
                ey = err_y(g.apply(op, x, prec), P.apply(op, x), absAx)
                record("err_y", prec, ey)
                assert ey <= tol, (alpha, op, ey)


def test_quad_points_leave_the_det_flag_alone():
    """sf_patch_quad_points evaluates G only: on a folded map it does not
    record a det J failure, so the next sf_patch_geometry_check (which reports
    the asynchronous prepares only) passes."""
    import torch
    kn, ctrl = inputs.identity_geometry((3, 3, 3), 3)
    folded = ctrl.copy()
    folded[:, 0] = -folded[:, 0]
    with GpuPatch(kn, 3, folded) as g:
        xyz = torch.empty((g.Q, 3), dtype=torch.float64, device="cuda")
        sf.sf_patch_quad_points(ctx(), g.h, xyz)
        sf.sf_patch_geometry_check(ctx(), g.h)         # SF_OK: no prepare ran
        assert float(xyz[:, 0].max()) <= 0.0           # the mirrored map was evaluated


def test_error_paths():
    kn, ctrl = inputs.identity_geometry((3, 3, 3), 3)
    folded = ctrl.copy()
    folded[:, 0] = -folded[:, 0]                    # mirrored map: det J < 0 everywhere
    with GpuPatch(kn, 3, folded) as g:
        with pytest.raises(sf.SfError) as e:
            g.prepare()
        assert e.value.status == sf.SF_EGEOM
    with GpuPatch(kn, 3, ctrl) as g:
        with pytest.raises(sf.SfError) as e:
            g.assemble(sf.SF_STIFF)                 # not prepared
        assert e.value.status == sf.SF_EINVAL
        with pytest.raises(sf.SfError) as e:
            g.prepare(prec=sf.SF_BF16_SPLIT + 7)
        assert e.value.status == sf.SF_EINVAL
        g.prepare(sf.SF_STIFF, sf.SF_FP16_SPLIT)
        with pytest.raises(sf.SfError) as e:
            g.assemble(sf.SF_STIFF, sf.SF_FP16_SPLIT)     # a storage of the apply only
        assert e.value.status == sf.SF_EUNSUPPORTED
        g.prepare(sf.SF_STIFF, sf.SF_BF16_SPLIT)
        with pytest.raises(sf.SfError) as e:
            g.apply(sf.SF_STIFF, np.ones(g.N), sf.SF_BF16_SPLIT)   # a mode of the assembly only
        assert e.value.status == sf.SF_EUNSUPPORTED
        g.prepare()
        assert g.assemble(sf.SF_STIFF).shape == (g.nnz,)     # still usable after errors
    # one order per direction in the descriptor; unequal orders are not built
    kn2 = [inputs.open_uniform_knots(3, 3), inputs.open_uniform_knots(3, 4), inputs.open_uniform_knots(3, 3)]
    with pytest.raises(sf.SfError) as e:
        sf.sf_patch_create(ctx(), 3, (3, 4, 3), kn2, np.zeros((5 * 6 * 5, 3)))
    assert e.value.status == sf.SF_EUNSUPPORTED
    with GpuPatch(kn, (3, 3, 3), ctrl) as g:       # equal orders given per direction
        g.prepare(sf.SF_STIFF)
    bad = [k.copy() for k in kn]
    bad[1][3], bad[1][4] = bad[1][4], bad[1][3]
    with pytest.raises(sf.SfError) as e:
        GpuPatch(bad, 3, ctrl)
    assert e.value.status == sf.SF_EKNOT


@pytest.mark.parametrize("K,p", [((5, 3, 4), 2), ((7, 5, 3), 3), ((20, 3, 2), 4), ((3, 4, 2), 6), ((2, 2, 1), 9),
                                 ((6,), 4), ((4, 5), 3)])
def test_eval_values_and_gradients(K, p):
    """sf_patch_eval (Algorithm 3 on the tensor grid of points, with the
    geometry's Jacobian in the same pass) against the oracle's plain sums
    over each point's active functions: values, physical gradients; and a
    linear physical function reproduced exactly (value and gradient)."""
    import torch
    d = len(K)
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=15)
    P = oracle.Problem(kn, p, ctrl)
    u = inputs.random_vector(P.N, 16)
    v_o, g_o, x_o = P.eval(u)
    with GpuPatch(kn, p, ctrl) as g:
        ud = torch.as_tensor(u).cuda()
        val = torch.full((g.Q,), float("nan"), dtype=torch.float64, device="cuda")
        grad = torch.full((g.Q, d), float("nan"), dtype=torch.float64, device="cuda")
        sf.sf_patch_eval(ctx(), g.h, ud, val, grad)
        torch.cuda.synchronize()
        ev = float(np.abs(val.cpu().numpy() - v_o).max() / np.abs(v_o).max())
        eg = float(np.abs(grad.cpu().numpy() - g_o).max() / np.abs(g_o).max())
        record("err_eval", sf.SF_FP64, max(ev, eg))
        assert ev <= TOL64 and eg <= TOL64, (ev, eg)
        # linear physical function gamma . x + beta: value and gradient exact
        gam = np.linspace(-0.8, 1.1, d)
        ul = torch.as_tensor(np.ascontiguousarray(ctrl.reshape(-1, d) @ gam + 0.5)).cuda()
        sf.sf_patch_eval(ctx(), g.h, ul, val, grad)
        torch.cuda.synchronize()
        assert np.abs(val.cpu().numpy() - (x_o @ gam + 0.5)).max() < 1e-12
        assert np.abs(grad.cpu().numpy() - gam[None, :]).max() < 1e-11
        # the physical points agree with sf_patch_quad_points
        xyz = torch.empty((g.Q, d), dtype=torch.float64, device="cuda")
        sf.sf_patch_quad_points(ctx(), g.h, xyz)
        torch.cuda.synchronize()
        assert np.abs(xyz.cpu().numpy() - x_o).max() < 1e-14


@pytest.mark.parametrize("policy", ["relabelled", "tune"])
@pytest.mark.parametrize("K,p", [((2, 9, 7), 3), ((8, 3, 6), 4), ((1, 12, 5), 2), ((6, 7, 2), 3)])
def test_contraction_order(monkeypatch, policy, K, p):
    """The assembly with the direction of fewest elements contracted last
    (the narrow direction last, Sec. 4.2): the patch is relabelled cyclically,
    assembled, and its values gathered into the given CSR layout.
    SFIGA_ASSEMBLY_ORDER=relabelled forces that path; by default the tuner
    times both orders and keeps the faster.  Full matrices and products
    against the oracle in FP64 and FP32; after a new coefficient and a new
    prepare the relabelled patch follows."""
    monkeypatch.setenv("SFIGA_ASSEMBLY_ORDER", policy)
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=17)
    _full_parity(kn, p, ctrl, ("sinprod", 0.5))
    _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_FP32, tol=TOL32)
    P2 = oracle.Problem(kn, p, ctrl, ("sinprod", -0.3))
    _, _, v_o = P2.assemble(sf.SF_STIFF)
    with GpuPatch(kn, p, ctrl, ("sinprod", 0.5)) as g:
        g.prepare(sf.SF_STIFF)
        g.assemble(sf.SF_STIFF)                               # tunes, creates the relabelled patch
        sf.sf_patch_set_coef(g.ctx, g.h, sf.SF_STIFF, sf.SF_COEF_SINPROD, -0.3)
        g.prepare(sf.SF_STIFF)
        v = g.assemble(sf.SF_STIFF)
        assert err_A(v, v_o) <= TOL64


@pytest.mark.parametrize("prec,tol", [(sf.SF_FP64, TOL64), (sf.SF_FP32, TOL32)])
def test_batched_apply_with_a_patch_applied_alone(prec, tol):
    """A batch patch whose own apply launch fills the chip (32 x 32 x 64
    elements at order 4, about 2k workgroups) runs its single-patch kernel on
    the tiled coefficient copy inside the captured batch call; the small
    patch beside it stays in the persistent kernel.  Sampled rows of the
    large patch and the whole small one against the oracle, on two calls."""
    import torch
    from tests.gpu_util import side_ctx
    c, stream = side_ctx()
    specs = [((32, 32, 64), 4, 3), ((4, 5, 3), 3, 4)]
    patches, probs, xs = [], [], []
    with torch.cuda.stream(stream):
        try:
            for K, p, seed in specs:
                kn, ctrl = inputs.perturbed_geometry(K, p, seed=seed, amp=0.05)
                g = GpuPatch(kn, p, ctrl, ("sinprod", 0.5), context=c)
                g.prepare(sf.SF_STIFF, prec)
                patches.append(g)
                probs.append(oracle.Problem(kn, p, ctrl, ("sinprod", 0.5)))
                xs.append(inputs.random_vector(g.N, seed))
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            ro, _ = sf.sf_batch_offsets(c, bt, 2)
            x = torch.as_tensor(np.concatenate(xs)).cuda()
            y = torch.empty(int(ro[-1]), dtype=torch.float64, device="cuda")
            rng = np.random.default_rng(5)
            rows = sample_rows(probs[0].nfun, rng, nrandom=8, coarse=True, p=4, band="cross")
            yref0 = probs[0].apply_rows_by_elements(oracle.STIFF, xs[0], rows)
            den0 = max(float(np.abs(v) @ np.abs(xs[0][cc])) for cc, v in probs[0].rows(oracle.STIFF, rows))
            rp, ci, v = probs[1].assemble(oracle.STIFF)
            A1 = oracle.csr_to_dense(rp, ci, v, probs[1].N)
            for rep in range(2):
                y.fill_(float("nan"))
                sf.sf_batch_apply(c, bt, sf.SF_STIFF, prec, x, y)
                stream.synchronize()
                yn = y.cpu().numpy()
                e0 = float(np.abs(yn[ro[0]:ro[1]][rows] - yref0).max() / den0)
                e1 = err_y(yn[ro[1]:ro[2]], A1 @ xs[1], np.abs(A1) @ np.abs(xs[1]))
                record("err_y", prec, max(e0, e1))
                assert e0 <= tol and e1 <= tol, (rep, e0, e1)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()
