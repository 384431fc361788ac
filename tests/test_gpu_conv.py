"""GPU parity of the convection form (SF_CONV, d = 3, FP64): the HIP kernel
pair through the C ABI against the oracle's convection form (op 4) on the
same seeded inputs.

Bar: err_y <= 1e-12, the FP64 bar of the other products (the sums are the
oracle's up to their order), with err_y = max |y - y_ref| / max (|B| |x|);
|B| |x| from the oracle's matrix where it is assembled whole, else from its
rows.  Large patches are checked on sampled rows (clipped bands, tile and
layer edges) and, at every row, through the identity B x_i = s b_i M 1 for
x_i the coefficients of the physical coordinate x_i, with M 1 from the
library's FP64 mass product."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_1809_05471_amd as sf
from paper_1809_05471_amd import inputs
from tests.gpu_util import COEF_KIND, ctx, record, sample_rows, torch_cuda

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


class ConvPatch:
    def __init__(self, knots, p, ctrl, coef, b):
        self.h = sf.sf_patch_create(ctx(), 3, p, knots, ctrl)
        self.N, self.nnz, self.Q = sf.sf_patch_info(self.h)
        kind, val = coef
        sf.sf_patch_set_coef(ctx(), self.h, sf.SF_CONV, COEF_KIND[kind], val)
        sf.sf_patch_set_convection(ctx(), self.h, b)

    def prepare(self, ops=sf.SF_CONV):
        sf.sf_patch_prepare(ctx(), self.h, ops, sf.SF_FP64)

    def apply(self, x, op=sf.SF_CONV):
        torch = torch_cuda()
        xd = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()
        y = torch.full((self.N,), float("nan"), dtype=torch.float64, device="cuda")
        sf.sf_apply(ctx(), self.h, op, sf.SF_FP64, xd, y)
        torch.cuda.synchronize()
        return y.cpu().numpy()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        sf.sf_patch_destroy(self.h)


def _full_check(K, p, coef, b, seed):
    # perturbation a fraction of the Greville spacing (about h / p), so that
    # the map stays regular at high orders
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=seed, amp=0.6 / p)
    P = oracle.Problem(kn, p, ctrl, coef, conv_b=b)
    rp, ci, v = P.assemble(oracle.CONV)
    A = sp.csr_matrix((v, ci, rp), shape=(P.N, P.N))
    x = inputs.random_vector(P.N, seed + 1)
    yref = A @ x
    den = np.abs(abs(A) @ np.abs(x)).max()
    with ConvPatch(kn, p, ctrl, coef, b) as g:
        g.prepare()
        y = g.apply(x)
        y2 = g.apply(x)                       # the point buffer is reused
    assert not np.isnan(y).any()
    e = float(np.abs(y - yref).max() / den)
    record("err_y", sf.SF_FP64, e)
    assert e <= TOL64, (K, p, e)
    assert float(np.abs(y2 - yref).max() / den) <= TOL64


# one tile and several (E = ceil(16 / p) elements per tile side), ragged
# edges, layers of one element
@pytest.mark.parametrize("K,p", [
    ((3, 4, 2), 2), ((9, 10, 3), 2), ((5, 3, 4), 3), ((7, 8, 2), 3), ((4, 4, 3), 4), ((5, 9, 2), 4),
    ((3, 5, 2), 5), ((5, 4, 1), 5), ((2, 3, 3), 6), ((4, 7, 2), 6), ((4, 2, 2), 7), ((2, 2, 3), 8),
    ((3, 5, 2), 8), ((3, 2, 2), 9), ((1, 1, 1), 4),
])
def test_conv_full_parity(K, p):
    _full_check(K, p, ("sinprod", 0.5), (0.7, -1.2, 0.4), seed=3 + p)


def test_conv_follows_a_new_vector_and_coefficient():
    K, p = (4, 5, 3), 4
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=8, amp=0.15)
    x = inputs.random_vector(int(np.prod([k + p - 1 for k in K])), 9)
    with ConvPatch(kn, p, ctrl, ("const", 1.0), (1.0, 0.0, 0.0)) as g:
        for coef, b in [(("const", 1.0), (1.0, 0.0, 0.0)), (("sinprod", -0.7), (0.0, 0.5, -2.0))]:
            sf.sf_patch_set_coef(ctx(), g.h, sf.SF_CONV, COEF_KIND[coef[0]], coef[1])
            sf.sf_patch_set_convection(ctx(), g.h, b)
            g.prepare()
            y = g.apply(x)
            P = oracle.Problem(kn, p, ctrl, coef, conv_b=b)
            yref = P.apply(oracle.CONV, x)
            assert np.abs(y - yref).max() <= TOL64 * np.abs(yref).max() * 10


def _sampled_check(K, p, seed, nrandom):
    coef, b = ("const", 1.3), (0.6, -0.9, 1.1)
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=seed, amp=0.05, interior_only=True)
    P = oracle.Problem(kn, p, ctrl, coef, conv_b=b)
    nfun = [k + p - 1 for k in K]
    rng = np.random.default_rng(seed)
    E = (16 + p - 1) // p
    # rows at the edges of the kernels' tiles (direction 1, 2) and layers
    edge = [(E * t + j, E * t + j, m3) for t in (1, 2) for j in (-1, 0, p - 2) for m3 in (0, p - 1, nfun[2] // 2)]
    rows = sample_rows(nfun, rng, nrandom=nrandom, coarse=True, p=p, extra=edge, band="cross")
    x = inputs.random_vector(P.N, seed + 1)
    with ConvPatch(kn, p, ctrl, coef, b) as g:
        sf.sf_patch_set_coef(ctx(), g.h, sf.SF_MASS, sf.SF_COEF_CONST, 1.0)
        g.prepare(sf.SF_CONV | sf.SF_MASS)
        y = g.apply(x)
        ones = g.apply(np.ones(P.N), op=sf.SF_MASS)
        ycoord = [g.apply(ctrl[:, i]) for i in range(3)]
    yref = P.apply_rows_by_elements(oracle.CONV, x, rows)
    absrow = np.array([np.abs(v) @ np.abs(x[c]) for c, v in P.rows(oracle.CONV, rows)])
    e = float(np.abs(y[rows] - yref).max() / absrow.max())
    record("err_y", sf.SF_FP64, e)
    assert e <= TOL64, e
    # every row: B x_i = s b_i M 1
    for i in range(3):
        ei = float(np.abs(ycoord[i] - coef[1] * b[i] * ones).max() / np.abs(ones).max())
        assert ei <= TOL64, (i, ei)


def test_conv_48cubed_p4_sampled_rows():
    _sampled_check((48, 48, 48), 4, seed=21, nrandom=24)


def test_conv_128cubed_p6_sampled_rows():
    _sampled_check((128, 128, 128), 6, seed=11, nrandom=12)


def test_conv_error_paths():
    K, p = (3, 3, 3), 3
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=4, amp=0.1)
    torch = torch_cuda()
    with ConvPatch(kn, p, ctrl, ("const", 1.0), (1.0, 1.0, 1.0)) as g:
        x = torch.zeros(g.N, dtype=torch.float64, device="cuda")
        y = torch.zeros(g.N, dtype=torch.float64, device="cuda")
        with pytest.raises(sf.SfError) as ei:
            sf.sf_apply(ctx(), g.h, sf.SF_CONV, sf.SF_FP64, x, y)        # not prepared
        assert ei.value.status == sf.SF_EINVAL
        for prec in (sf.SF_FP32, sf.SF_FP16_SPLIT):
            with pytest.raises(sf.SfError) as ei:
                sf.sf_patch_prepare(ctx(), g.h, sf.SF_CONV, prec)
            assert ei.value.status == sf.SF_EUNSUPPORTED
        g.prepare()
        with pytest.raises(sf.SfError) as ei:
            sf.sf_apply(ctx(), g.h, sf.SF_CONV, sf.SF_FP32, x, y)
        assert ei.value.status == sf.SF_EUNSUPPORTED
        v = torch.zeros(g.nnz, dtype=torch.float64, device="cuda")
        with pytest.raises(sf.SfError) as ei:
            sf.sf_assemble(ctx(), g.h, sf.SF_CONV, sf.SF_FP64, val_mass=v, val_stiff=v)
        assert ei.value.status == sf.SF_EUNSUPPORTED
        with pytest.raises(sf.SfError) as ei:
            sf.sf_apply(ctx(), g.h, sf.SF_CONV, sf.SF_FP64, x, x)
        assert ei.value.status == sf.SF_EINVAL
        # a new vector needs a new prepare
        sf.sf_patch_set_convection(ctx(), g.h, (0.0, 1.0, 0.0))
        with pytest.raises(sf.SfError) as ei:
            sf.sf_apply(ctx(), g.h, sf.SF_CONV, sf.SF_FP64, x, y)
        assert ei.value.status == sf.SF_EINVAL
    kn2, ctrl2 = inputs.perturbed_geometry((3, 3), 3, seed=4, amp=0.1)
    h2 = sf.sf_patch_create(ctx(), 2, 3, kn2, ctrl2)
    try:
        with pytest.raises(sf.SfError) as ei:
            sf.sf_patch_prepare(ctx(), h2, sf.SF_CONV, sf.SF_FP64)
        assert ei.value.status == sf.SF_EUNSUPPORTED
    finally:
        sf.sf_patch_destroy(h2)


def test_conv_qp_values_coefficient_matches_builtin():
    """SF_COEF_QPVALUES for the convection factor s, fed with the built-in
    sinprod at sf_patch_quad_points, gives the built-in product."""
    import torch
    K, p = (5, 4, 3), 4
    kn, ctrl = inputs.perturbed_geometry(K, p, seed=9, amp=0.1)
    x = inputs.random_vector(int(np.prod([k + p - 1 for k in K])), 2)
    with ConvPatch(kn, p, ctrl, ("sinprod", 0.5), (0.3, 1.0, -0.4)) as g:
        g.prepare()
        ref = g.apply(x)
        xyz = torch.empty((g.Q, 3), dtype=torch.float64, device="cuda")
        sf.sf_patch_quad_points(ctx(), g.h, xyz)
        s = (1.0 + 0.5 * torch.prod(torch.sin(2 * np.pi * xyz), dim=1)).contiguous()
        sf.sf_patch_set_coef(ctx(), g.h, sf.SF_CONV, sf.SF_COEF_QPVALUES, qp_values=s)
        g.prepare()
        y = g.apply(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
