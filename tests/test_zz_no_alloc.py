"""sf_assemble_noalloc (the assembly entry point that allocates nothing, for
callers that cannot call hipMalloc): through the C ABI, against sf_assemble
on the same prepared patches, to the FP64 bar (1e-12 of max |A|; the two
differ only in the summation order of entries that straddle a chunk of the
fixed scratch).  Two calls in a row, the second on a smaller patch, so that
the second runs on what the first left in the shared scratch; a patch too
large for the scratch is refused with SF_EUNSUPPORTED."""
import numpy as np
import pytest

import paper_1809_05471_amd as sf
from paper_1809_05471_amd import inputs
from tests.gpu_util import GpuPatch, ctx, err_A

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _both(g, ops, prec):
    import torch
    out = {}
    for op in (sf.SF_MASS, sf.SF_STIFF):
        if not ops & op:
            continue
        ref = torch.full((g.nnz,), float("nan"), dtype=torch.float64, device="cuda")
        got = torch.full((g.nnz,), float("nan"), dtype=torch.float64, device="cuda")
        kw = "val_mass" if op == sf.SF_MASS else "val_stiff"
        sf.sf_assemble(ctx(), g.h, op, prec, **{kw: ref})
        sf.sf_assemble_noalloc(ctx(), g.h, op, prec, **{kw: got})
        torch.cuda.synchronize()
        out[op] = (ref.cpu().numpy(), got.cpu().numpy())
    return out


def test_noalloc_matches_sf_assemble_two_calls():
    # first call: 48^3 order 4, stiffness and mass; the stiffness partials
    # (0.40 GB) run in two chunks of the 256 MiB scratch
    w = inputs.workload_3d((48, 48, 48), 4)
    with GpuPatch(w["knots"], 4, w["ctrl"], w["coef"]) as g:
        g.prepare(sf.SF_MASS | sf.SF_STIFF, sf.SF_FP64)
        for op, (ref, got) in _both(g, sf.SF_MASS | sf.SF_STIFF, sf.SF_FP64).items():
            assert not np.isnan(got).any(), op
            assert err_A(got, ref) <= TOL64, (op, err_A(got, ref))
    # second call, smaller patch and another order, in FP64 and FP32
    kn, ctrl = inputs.perturbed_geometry((9, 7, 11), 3, seed=21)
    with GpuPatch(kn, 3, ctrl, ("sinprod", 0.5)) as g:
        for prec, tol in ((sf.SF_FP64, TOL64), (sf.SF_FP32, 0.0)):
            g.prepare(sf.SF_MASS | sf.SF_STIFF, prec)
            for op, (ref, got) in _both(g, sf.SF_MASS | sf.SF_STIFF, prec).items():
                assert not np.isnan(got).any(), op
                # one chunk here: the same kernels and tiles, so the same bits
                assert err_A(got, ref) <= max(tol, 1e-15), (prec, op, err_A(got, ref))


def test_noalloc_refuses_a_patch_larger_than_the_scratch():
    # 200 x 200 x 4 elements at order 4: three element layers of stiffness
    # partials are 0.40 GB, above the 256 MiB scratch
    kn, ctrl = inputs.perturbed_geometry((200, 200, 4), 4, seed=22)
    with GpuPatch(kn, 4, ctrl) as g:
        g.prepare(sf.SF_STIFF, sf.SF_FP64)
        import torch
        v = torch.empty(g.nnz, dtype=torch.float64, device="cuda")
        with pytest.raises(sf.SfError) as e:
            sf.sf_assemble_noalloc(ctx(), g.h, sf.SF_STIFF, sf.SF_FP64, val_stiff=v)
        assert e.value.status == sf.SF_EUNSUPPORTED
        # the mass partials are a quarter of that and fit
        g.prepare(sf.SF_MASS, sf.SF_FP64)
        ref = torch.empty(g.nnz, dtype=torch.float64, device="cuda")
        sf.sf_assemble(ctx(), g.h, sf.SF_MASS, sf.SF_FP64, val_mass=ref)
        sf.sf_assemble_noalloc(ctx(), g.h, sf.SF_MASS, sf.SF_FP64, val_mass=v)
        torch.cuda.synchronize()
        assert err_A(v.cpu().numpy(), ref.cpu().numpy()) <= TOL64
