"""GPU parity of the glued multipatch product sf_batch_apply_glued
(Sec. 4, Example "Multipatch domains"): conforming d = 3 patches cut from a
patch with C0 interior knots, glued with the library's sf_glue_map; y
against the oracle's product on the C0 patch (the same operator, see
tests/test_oracle_glue.py), FP64 and FP32 at the bars of the other
products, on the default stream and on a side stream (captured graph,
replayed)."""
import numpy as np
import pytest

import oracle
import paper_1809_05471_amd as sf
from paper_1809_05471_amd import inputs
from tests.gpu_util import GpuPatch, ctx, err_y, record, side_ctx
from tests.test_oracle_glue import c0_split, interfaces_of

pytestmark = pytest.mark.gpu

TOL = {sf.SF_FP64: 1e-12, sf.SF_FP32: 1e-6}


@pytest.mark.parametrize("K,splits,p,prec,side", [
    ((6, 4, 3), ((3, 3), (2, 2), (3,)), 2, sf.SF_FP64, False),
    ((5, 6, 4), ((2, 3), (3, 3), (1, 3)), 3, sf.SF_FP64, True),
    ((8, 4, 4), ((3, 5), (4,), (2, 2)), 4, sf.SF_FP64, True),
    ((6, 6, 3), ((3, 3), (2, 4), (3,)), 6, sf.SF_FP64, False),
    ((5, 6, 4), ((2, 3), (3, 3), (1, 3)), 3, sf.SF_FP32, True),
    ((4, 4, 4), ((2, 2), (2, 2), (2, 2)), 5, sf.SF_FP32, False),
])
def test_glued_apply_equals_c0_patch(K, splits, p, prec, side):
    import torch
    c, stream = side_ctx() if side else (ctx(), torch.cuda.current_stream())
    coef = ("sinprod", 0.4)
    kn0, ctrl0, pieces = c0_split(K, splits, p, seed=11)
    single = oracle.Problem(kn0, p, ctrl0, coef)
    nf = [pc[2] for pc in pieces]
    m, ng = sf.sf_glue_map(3, nf, interfaces_of(splits))
    assert ng == single.N
    # the glued numbering as a relabelling of the C0 patch's functions
    perm = np.full(ng, -1)
    offs = np.cumsum([0] + [int(np.prod(n)) for n in nf])
    for b, pc in enumerate(pieces):
        perm[m[offs[b]:offs[b + 1]]] = pc[3]
    assert sorted(perm.tolist()) == list(range(ng))
    x = inputs.random_vector(ng, 5)
    xc0 = np.zeros(ng)
    xc0[perm] = x
    patches = []
    with torch.cuda.stream(stream):
        try:
            for kn, cc, _, _ in pieces:
                g = GpuPatch(kn, p, cc, coef, context=c)
                g.prepare(prec=prec)
                patches.append(g)
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            dmap = torch.as_tensor(m).cuda()
            xd = torch.as_tensor(x).cuda()
            y = torch.empty(ng, dtype=torch.float64, device="cuda")
            for op in (sf.SF_MASS, sf.SF_STIFF):
                rp, ci, v = single.assemble(op)
                A = np.zeros((ng, ng))
                for r in range(ng):
                    A[r, ci[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
                yref = (A @ xc0)[perm]
                absAx = (np.abs(A) @ np.abs(xc0))[perm]
                for rep in range(2):                 # capture, then replay on a side stream
                    y.fill_(float("nan"))
                    sf.sf_batch_apply_glued(c, bt, op, prec, dmap, ng, xd, y)
                    stream.synchronize()
                    e = err_y(y.cpu().numpy(), yref, absAx)
                    record("err_y", prec, e)
                    assert e <= TOL[prec], (op, rep, e)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()


def test_glued_apply_errors():
    import torch
    kn0, ctrl0, pieces = c0_split((4, 2, 2), ((2, 2), (2,), (2,)), 3, seed=2)
    patches = [GpuPatch(kn, 3, cc) for kn, cc, _, _ in pieces]
    try:
        for g in patches:
            g.prepare()
        bt = sf.sf_batch_create(ctx(), [g.h for g in patches])
        m, ng = sf.sf_glue_map(3, [pc[2] for pc in pieces], interfaces_of(((2, 2), (2,), (2,))))
        dmap = torch.as_tensor(m).cuda()
        x = torch.zeros(ng, dtype=torch.float64, device="cuda")
        with pytest.raises(sf.SfError) as ei:
            sf.sf_batch_apply_glued(ctx(), bt, sf.SF_STIFF, sf.SF_FP64, dmap, ng, x, x)
        assert ei.value.status == sf.SF_EINVAL
        with pytest.raises(sf.SfError) as ei:
            sf.sf_batch_apply_glued(ctx(), bt, sf.SF_STIFF, sf.SF_FP32, dmap, ng, x,
                                    torch.zeros(ng, dtype=torch.float64, device="cuda"))
        assert ei.value.status == sf.SF_EINVAL                   # FP32 not prepared
        sf.sf_batch_destroy(bt)
    finally:
        for g in patches:
            g.close()


def test_two_glued_groups_of_different_orders_in_one_batch():
    """Pieces of two C0 patches (orders 3 and 5) in one batch: the glued map
    is block-diagonal between the groups and the persistent launches mix
    the orders; each group against the oracle's C0 patch."""
    import torch
    c, stream = side_ctx()
    groups = [((4, 4, 3), ((2, 2), (4,), (3,)), 3), ((4, 3, 4), ((2, 2), (3,), (1, 3)), 5)]
    built, nf, ifc = [], [], []
    for K, splits, p in groups:
        kn0, ctrl0, pieces = c0_split(K, splits, p, seed=4)
        base = len(nf)
        ifc += [(a + base, fa, b + base, fb) for a, fa, b, fb in interfaces_of(splits)]
        nf += [pc[2] for pc in pieces]
        built.append((kn0, ctrl0, pieces, p))
    m, ng = sf.sf_glue_map(3, nf, ifc)
    offs = np.cumsum([0] + [int(np.prod(n)) for n in nf])
    patches = []
    with torch.cuda.stream(stream):
        try:
            for kn0, ctrl0, pieces, p in built:
                for kn, cc, _, _ in pieces:
                    g = GpuPatch(kn, p, cc, ("sinprod", 0.4), context=c)
                    g.prepare()
                    patches.append(g)
            bt = sf.sf_batch_create(c, [g.h for g in patches])
            x = inputs.random_vector(ng, 8)
            dmap = torch.as_tensor(m).cuda()
            y = torch.empty(ng, dtype=torch.float64, device="cuda")
            for rep in range(2):
                y.fill_(float("nan"))
                sf.sf_batch_apply_glued(c, bt, sf.SF_STIFF, sf.SF_FP64, dmap, ng, torch.as_tensor(x).cuda(), y)
                stream.synchronize()
                yn = y.cpu().numpy()
                b = 0
                for kn0, ctrl0, pieces, p in built:
                    single = oracle.Problem(kn0, p, ctrl0, ("sinprod", 0.4))
                    perm = {}
                    for pc in pieces:
                        for gid, c0 in zip(m[offs[b]:offs[b + 1]], pc[3]):
                            perm[int(gid)] = int(c0)
                        b += 1
                    gids = np.array(sorted(perm))
                    c0i = np.array([perm[i] for i in gids])
                    assert len(gids) == single.N
                    xc0 = np.zeros(single.N)
                    xc0[c0i] = x[gids]
                    yc0 = single.apply(oracle.STIFF, xc0)
                    rp, ci, v = single.assemble(oracle.STIFF)
                    absAx = np.array([np.abs(v[rp[r]:rp[r + 1]]) @ np.abs(xc0[ci[rp[r]:rp[r + 1]]])
                                      for r in range(single.N)])
                    e = err_y(yn[gids], yc0[c0i], absAx[c0i])
                    record("err_y", sf.SF_FP64, e)
                    assert e <= TOL[sf.SF_FP64], (rep, p, e)
            sf.sf_batch_destroy(bt)
        finally:
            for g in patches:
                g.close()
