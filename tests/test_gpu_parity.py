"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP64 bar (the paper: sum factorization gives the standard matrix up to
machine precision): err_A <= 1e-12 and err_y <= 1e-12, metrics in
tests/gpu_util.py.  FP32 mode: err <= 2e-5 (the coefficient tensor and the
contractions round to 2^-24; sums of O(p^2) terms per level, three levels).
Patterns and row pointers are compared bit-exactly.
"""
import numpy as np
import pytest

import oracle
import paper_1809_05471_amd as sf
from paper_1809_05471_amd import inputs
from tests.gpu_util import GpuPatch, ctx, err_A, err_y, sample_rows

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5
# BF16 split: operands x = hi + lo in bf16 hold x to 2^-17; a product keeps
# Ahi Bhi + Ahi Blo + Alo Bhi (dropping Alo Blo ~ 2^-18), so each level-2
# term carries about 2^-16 relative error before the FP32 and FP64 sums
TOLBF = 2e-4


def _full_parity(knots, p, ctrl, coef, ops=(sf.SF_MASS, sf.SF_STIFF), prec=sf.SF_FP64, tol=TOL64, seed=0):
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
            v = g.assemble(op, prec)
            assert not np.isnan(v).any()
            eA = err_A(v, v_o)
            A = oracle.csr_to_dense(rp_o, ci_o, v_o, P.N) if P.N <= 4000 else None
            y_o = P.apply(op, x)
            y = g.apply(op, x, prec)
            absAx = np.abs(A) @ np.abs(x) if A is not None else None
            if absAx is None:
                absAx = np.zeros(P.N)
                np.add.at(absAx, np.repeat(np.arange(P.N), np.diff(rp_o)), np.abs(v_o) * np.abs(x[ci_o]))
            ey = err_y(y, y_o, absAx)
            assert eA <= tol, (op, eA)
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
    checked against the FP64 oracle with the bound TOLBF."""
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=4)
    res = _full_parity(kn, p, ctrl, ("sinprod", 0.5), prec=sf.SF_BF16_SPLIT, tol=TOLBF)
    # the split keeps far more than bf16 alone (2^-9 ~ 2e-3) would
    assert max(eA for eA, _ in res.values()) < 1e-4


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


def _sampled_parity(w, ops, prec=sf.SF_FP64, tol=TOL64, nrandom=48, assemble=True, coarse=False):
    kn, p, ctrl, coef, x = w["knots"], w["p"], w["ctrl"], w["coef"], w["x"]
    P = oracle.Problem(kn, p, ctrl, coef)
    rows = sample_rows(P.nfun, np.random.default_rng(5), nrandom, coarse)
    res = {}
    with GpuPatch(kn, p, ctrl, coef) as g:
        g.prepare(prec=prec)
        if assemble:
            rp, ci = g.pattern()
            assert rp[-1] == g.nnz
        for op in ops:
            ref = P.rows(op, rows)
            vmax = max(np.abs(v).max() for _, v in ref)
            absAx = np.array([np.abs(v) @ np.abs(x[c]) for c, v in ref])
            if assemble:
                vals = g.assemble(op, prec)
                worst = 0.0
                for r, (c, v) in zip(rows, ref):
                    cg = ci[rp[r]:rp[r + 1]]
                    assert np.array_equal(cg.astype(np.int64), c)
                    worst = max(worst, float(np.abs(vals[rp[r]:rp[r + 1]] - v).max()))
                assert worst / vmax <= tol, (op, worst / vmax)
                res[("A", op)] = worst / vmax
            y = g.apply(op, x, prec)
            y_o = P.apply_rows(op, x, rows)
            ey = float(np.abs(y[rows] - y_o).max() / absAx.max())
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


@pytest.mark.parametrize("prec,tol", [(sf.SF_FP64, TOL64), (sf.SF_FP32, TOL32)])
def test_3d_128cubed_p6_sampled_rows(prec, tol):
    """Large patch: d = 3, 128^3 elements, order 6 (N = 2,352,637, nnz =
    2,942,649,737), perturbed geometry, a = 1 + 0.5 sin sin sin; stiffness
    assembly (in chunks of element layers) and y = A x, compared with the
    oracle on sampled rows; only those rows leave the device."""
    import torch
    w = inputs.workload_3d((128, 128, 128), 6)
    kn, p, ctrl, coef, x = w["knots"], w["p"], w["ctrl"], w["coef"], w["x"]
    P = oracle.Problem(kn, p, ctrl, coef)
    rows = sample_rows(P.nfun, np.random.default_rng(11), 12, coarse=True)
    ref = P.rows(sf.SF_STIFF, rows)
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
        worst = 0.0
        for r, (c, vr) in zip(rows, ref):
            a, b = int(rpn[r]), int(rpn[r + 1])
            assert np.array_equal(ci[a:b].cpu().numpy().astype(np.int64), c)
            worst = max(worst, float(np.abs(v[a:b].cpu().numpy() - vr).max()))
        assert worst / vmax <= tol, worst / vmax
        del v, ci
        y = g.apply(sf.SF_STIFF, x, prec)
        absAx = np.array([np.abs(vr) @ np.abs(x[c]) for c, vr in ref])
        ey = float(np.abs(y[rows] - P.apply_rows(sf.SF_STIFF, x, rows)).max() / absAx.max())
        assert ey <= tol, ey
        # K 1 = 0 on every row (partition of unity), through the matrix-free path
        y1 = g.apply(sf.SF_STIFF, np.ones(g.N), prec)
        assert np.abs(y1).max() <= (1e-12 if prec == sf.SF_FP64 else 1e-5) * vmax


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8, 9])
def test_order_sweep_apply_sampled(p):
    """d = 3, K = 127 - p per direction (N = 126^3 for every order), matrix-free
    stiffness apply on sampled rows, FP64 and FP32."""
    w = inputs.workload_order_sweep(p)
    coarse = p >= 6
    _sampled_parity(w, (sf.SF_STIFF,), nrandom=4 if coarse else 16, assemble=False, coarse=coarse)
    if p in (4, 6):
        _sampled_parity(w, (sf.SF_STIFF,), prec=sf.SF_FP32, tol=TOL32, nrandom=4, assemble=False, coarse=True)


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
        with pytest.raises(sf.SfError) as e:
            g.prepare(prec=sf.SF_FP16_SPLIT)
        assert e.value.status == sf.SF_EUNSUPPORTED
        g.prepare()
        assert g.assemble(sf.SF_STIFF).shape == (g.nnz,)     # still usable after errors
    bad = [k.copy() for k in kn]
    bad[1][3], bad[1][4] = bad[1][4], bad[1][3]
    with pytest.raises(sf.SfError) as e:
        GpuPatch(bad, 3, ctrl)
    assert e.value.status == sf.SF_EKNOT
