"""Helpers for the GPU parity tests: a small wrapper that drives the C ABI
through the Python binding (torch for device buffers) and the error metrics
used against the oracle:
  err_A = max |A - A_ref| / max |A_ref|
  err_y = max |y - y_ref| / max (|A_ref| |x|)
"""
import numpy as np

import paper_1809_05471_amd as sf

_CTX = None
_SIDE = None


def torch_cuda():
    import torch
    return torch


def ctx():
    global _CTX
    if _CTX is None:
        torch = torch_cuda()
        torch.cuda.init()
        _CTX = sf.sf_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    return _CTX


def side_ctx():
    """A second context on a torch side stream (default priority): its
    batched calls are captured into HIP graphs and replayed."""
    global _SIDE
    if _SIDE is None:
        torch = torch_cuda()
        torch.cuda.init()
        stream = torch.cuda.Stream()
        _SIDE = (sf.sf_ctx_create(0, stream.cuda_stream), stream)
    return _SIDE


COEF_KIND = {"const": sf.SF_COEF_CONST, "sinprod": sf.SF_COEF_SINPROD}


class GpuPatch:
    def __init__(self, knots, p, ctrl, coef=("const", 1.0), context=None):
        self.d = len(knots)
        self.p = p
        self.ctx = context if context is not None else ctx()
        self.h = sf.sf_patch_create(self.ctx, self.d, p, knots, ctrl)
        self.N, self.nnz, self.Q = sf.sf_patch_info(self.h)
        kind, val = coef
        sf.sf_patch_set_coef(self.ctx, self.h, sf.SF_STIFF, COEF_KIND[kind], val)

    def prepare(self, ops=sf.SF_MASS | sf.SF_STIFF, prec=sf.SF_FP64):
        sf.sf_patch_prepare(self.ctx, self.h, ops, prec)

    def pattern(self):
        torch = torch_cuda()
        rp = torch.empty(self.N + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        sf.sf_csr_pattern(ctx(), self.h, rp, ci)
        torch.cuda.synchronize()
        return rp.cpu().numpy(), ci.cpu().numpy()

    def assemble(self, op, prec=sf.SF_FP64, keep_on_device=False):
        torch = torch_cuda()
        v = torch.full((self.nnz,), float("nan"), dtype=torch.float64, device="cuda")
        if op == sf.SF_MASS:
            sf.sf_assemble(ctx(), self.h, op, prec, val_mass=v)
        else:
            sf.sf_assemble(ctx(), self.h, op, prec, val_stiff=v)
        torch.cuda.synchronize()
        return v if keep_on_device else v.cpu().numpy()

    def apply(self, op, x, prec=sf.SF_FP64):
        torch = torch_cuda()
        xd = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()
        y = torch.full((self.N,), float("nan"), dtype=torch.float64, device="cuda")
        sf.sf_apply(ctx(), self.h, op, prec, xd, y)
        torch.cuda.synchronize()
        return y.cpu().numpy()

    def close(self):
        if self.h:
            sf.sf_patch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def err_A(v, vref):
    return float(np.abs(v - vref).max() / np.abs(vref).max())


def err_y(y, yref, absAx):
    return float(np.abs(y - yref).max() / np.abs(absAx).max())


def sample_rows(nfun, rng, nrandom=64, coarse=False):
    """Corner, edge, face and interior rows of a tensor grid plus random ones
    (coarse: only first / middle / last index per direction)."""
    d = len(nfun)
    picks = set()
    choices = [[0, n // 2, n - 1] if coarse else [0, 1, n // 2, n - 2, n - 1] for n in nfun]
    grids = np.meshgrid(*choices, indexing="ij")
    for idx in zip(*[g.ravel() for g in grids]):
        m, stride = 0, 1
        for k in range(d):
            m += int(idx[k]) * stride
            stride *= nfun[k]
        picks.add(m)
    N = int(np.prod(nfun))
    picks.update(int(v) for v in rng.integers(0, N, nrandom))
    return np.array(sorted(picks), dtype=np.int64)
