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


# measured errors of the session: (test, quantity, precision, value), printed
# in the terminal summary (tests/conftest.py) so that the bounds can be set
# from measurements
MEASURED = []

PREC_NAME = {sf.SF_FP64: "fp64", sf.SF_FP32: "fp32", sf.SF_BF16_SPLIT: "bf16_split",
             sf.SF_FP16_SPLIT: "fp16_split"}


def record(what, prec, value):
    import os
    MEASURED.append((os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0], what,
                     PREC_NAME.get(prec, str(prec)), float(value)))


def err_A(v, vref):
    return float(np.abs(v - vref).max() / np.abs(vref).max())


def err_y(y, yref, absAx):
    return float(np.abs(y - yref).max() / np.abs(absAx).max())


def _lin(idx, nfun):
    m, stride = 0, 1
    for k in range(len(nfun)):
        m += int(idx[k]) * stride
        stride *= nfun[k]
    return m


def sample_rows(nfun, rng, nrandom=64, coarse=False, p=None, extra=(), band="grid"):
    """Corner, edge, face and interior rows of a tensor grid plus random ones
    (coarse: only first / middle / last index per direction).  With the order
    p, the indices 1, p-2, N-p+1 and N-2 are added in every direction: rows
    whose 1D band (Corollary on #NZ) is clipped by the boundary; band="grid"
    takes every combination, band="cross" varies one direction at a time
    (the others at their first / middle / last index).  `extra` is a list of
    multi-indices (direction 1 first) added as they are."""
    d = len(nfun)
    picks = set()
    base, clipped = [], []
    for n in nfun:
        c = {0, n // 2, n - 1} if coarse else {0, 1, n // 2, n - 2, n - 1}
        base.append(sorted(v for v in c if 0 <= v < n))
        clipped.append(sorted(v for v in {1, p - 2, n - p + 1, n - 2} if 0 <= v < n) if p is not None else [])
    if band == "grid":
        sets = [[sorted(set(base[k]) | set(clipped[k])) for k in range(d)]]
    else:
        sets = [base] + [[clipped[k] if k == j else base[k] for k in range(d)] for j in range(d)]
    for choices in sets:
        grids = np.meshgrid(*choices, indexing="ij")
        for idx in zip(*[g.ravel() for g in grids]):
            picks.add(_lin(idx, nfun))
    for idx in extra:
        if all(0 <= int(idx[k]) < nfun[k] for k in range(d)):
            picks.add(_lin(idx, nfun))
    N = int(np.prod(nfun))
    picks.update(int(v) for v in rng.integers(0, N, nrandom))
    return np.array(sorted(picks), dtype=np.int64)


def half_windows(p):
    """Stored level-2 windows per (m1, m2) of the library's assembly: the
    upper half of the (2p-1)^2 band windows, used to predict its chunks."""
    return (p - 1) * (2 * p - 1) + p


def chunk_boundaries(nfun, nel, p, prec_bytes, ops_groups=4, cap_mb=4096, sized_bytes=8):
    """Direction-3 element layers where the library's level-1/2 workspace is
    split into chunks (its rule: the workspace holds as many whole element
    layers of level-2 partials as fit in the cap, sized for FP64 stiffness;
    a precision with smaller partials fits proportionally more layers).
    Returns the first layer s0 > 0 of every chunk."""
    plane = ops_groups * nfun[1] * nfun[0] * half_windows(p)
    per_layer_sized = plane * sized_bytes * p
    K3 = nel[2]
    layers = min(max((cap_mb << 20) // per_layer_sized, max(p - 1, 1)), K3)
    ws = layers * per_layer_sized
    chunk = min(ws // (plane * prec_bytes * p), K3)
    return list(range(chunk, K3, chunk))


def straddle_rows(nfun, nel, p, prec_bytes, picks_12):
    """Rows m = (m1, m2, m3) with m3 in [s0, s0 + p - 2] for every chunk
    boundary s0: their entries with n3 in the same range collect level-3
    sums from both sides of the boundary."""
    out = []
    for s0 in chunk_boundaries(nfun, nel, p, prec_bytes):
        for m3 in range(s0, min(s0 + p - 1, nfun[2])):
            for m1, m2 in picks_12:
                out.append((m1, m2, m3))
    return out
