"""sfiga: sum-factorized isogeometric assembly and matrix-free apply on MI355X.

Thin ctypes binding over the C ABI in ``include/sfiga.h`` (``libsfiga.so``,
built in-tree by ``paper_1809_05471_amd.build``).  Every function below has
the name of the C entry point it marshals to; device buffers are passed as
torch tensors (their ``data_ptr()``) or raw integer addresses.  All compute
runs in the HIP library: if it is missing the import of the library raises.
"""
from __future__ import annotations

import ctypes
import os
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfiga.so")

SF_OK, SF_EINVAL, SF_EKNOT, SF_EGEOM, SF_ENOMEM, SF_EDEVICE, SF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SF_FP64, SF_FP32, SF_BF16_SPLIT, SF_FP16_SPLIT = 0, 1, 2, 3
SF_MASS, SF_STIFF, SF_CONV = 1, 2, 4
SF_COEF_CONST, SF_COEF_SINPROD, SF_COEF_QPVALUES = 0, 1, 2

STATUS_NAMES = {0: "SF_OK", -1: "SF_EINVAL", -2: "SF_EKNOT", -3: "SF_EGEOM", -4: "SF_ENOMEM",
                -5: "SF_EDEVICE", -6: "SF_EUNSUPPORTED"}

EXPORTED = ["sf_ctx_create", "sf_ctx_destroy", "sf_last_error", "sf_build_target", "sf_host_tables_1d",
            "sf_patch_create",
            "sf_patch_info", "sf_patch_set_coef", "sf_patch_set_convection", "sf_patch_set_diffusion", "sf_patch_quad_points", "sf_patch_eval", "sf_patch_prepare",
            "sf_patch_prepare_async", "sf_patch_geometry_check", "sf_csr_pattern", "sf_assemble", "sf_assemble_noalloc", "sf_apply", "sf_patch_destroy", "sf_batch_create",
            "sf_batch_offsets", "sf_batch_assemble", "sf_batch_apply", "sf_glue_map", "sf_batch_apply_glued",
            "sf_batch_destroy"]


class SfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class PatchDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("order", ctypes.c_int * 3), ("n_knots", ctypes.c_int64 * 3),
                ("knots", ctypes.POINTER(ctypes.c_double) * 3), ("ctrl", ctypes.c_void_p),
                ("ctrl_on_device", ctypes.c_int)]


@lru_cache(maxsize=1)
def lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1809_05471_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    st = ctypes.c_int
    sig = {
        "sf_ctx_create": (st, [ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "sf_ctx_destroy": (None, [vp]),
        "sf_last_error": (ctypes.c_char_p, [vp]),
        "sf_build_target": (ctypes.c_char_p, []),
        "sf_host_tables_1d": (st, [vp, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_int), vp, vp, vp,
                                   vp]),
        "sf_patch_create": (st, [vp, ctypes.POINTER(PatchDesc), ctypes.POINTER(vp)]),
        "sf_patch_info": (st, [vp, i64p, i64p, i64p]),
        "sf_patch_set_coef": (st, [vp, ctypes.c_uint, ctypes.c_int, vp]),
        "sf_patch_set_convection": (st, [vp, vp]),
        "sf_patch_set_diffusion": (st, [vp, vp]),
        "sf_patch_quad_points": (st, [vp, vp]),
        "sf_patch_eval": (st, [vp, vp, vp, vp]),
        "sf_patch_prepare": (st, [vp, ctypes.c_uint, ctypes.c_int]),
        "sf_patch_prepare_async": (st, [vp, ctypes.c_uint, ctypes.c_int]),
        "sf_patch_geometry_check": (st, [vp]),
        "sf_csr_pattern": (st, [vp, vp, vp]),
        "sf_assemble": (st, [vp, ctypes.c_uint, ctypes.c_int, vp, vp]),
        "sf_assemble_noalloc": (st, [vp, ctypes.c_uint, ctypes.c_int, vp, vp]),
        "sf_apply": (st, [vp, ctypes.c_uint, ctypes.c_int, vp, vp]),
        "sf_patch_destroy": (None, [vp]),
        "sf_batch_create": (st, [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "sf_batch_offsets": (st, [vp, i64p, i64p]),
        "sf_batch_assemble": (st, [vp, ctypes.c_uint, ctypes.c_int, vp, vp, vp, vp]),
        "sf_batch_apply": (st, [vp, ctypes.c_uint, ctypes.c_int, vp, vp]),
        "sf_glue_map": (st, [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp, vp, i64p]),
        "sf_batch_apply_glued": (st, [vp, ctypes.c_uint, ctypes.c_int, vp, ctypes.c_int64, vp, vp]),
        "sf_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _ptr(t):
    """Device address of a torch tensor (or an int / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _check(status, ctx):
    if status != SF_OK:
        msg = lib().sf_last_error(ctx).decode() if ctx else ""
        raise SfError(status, msg)


# ------------------------------------------------------------ C entry points

def sf_build_target():
    return lib().sf_build_target().decode()


def sf_host_tables_1d(knots, order):
    """Host-side 1D tables (points, weights, values, derivatives) of one direction."""
    t = np.ascontiguousarray(knots, dtype=np.float64)
    K = max(len(t) - 2 * order + 1, 0)
    x = np.zeros((K, order))
    w = np.zeros((K, order))
    B = np.zeros((K, order, order))
    D = np.zeros((K, order, order))
    nel = ctypes.c_int(0)
    st = lib().sf_host_tables_1d(t.ctypes.data, len(t), order, ctypes.byref(nel), x.ctypes.data, w.ctypes.data,
                                 B.ctypes.data, D.ctypes.data)
    if st != SF_OK:
        raise SfError(st, "invalid knot vector")
    return dict(nel=nel.value, x=x, w=w, B=B, D=D)


def sf_ctx_create(device=0, stream=None):
    out = ctypes.c_void_p()
    st = lib().sf_ctx_create(device, stream, ctypes.byref(out))
    if st != SF_OK:
        raise SfError(st, "context creation failed")
    return out.value


def sf_ctx_destroy(ctx):
    lib().sf_ctx_destroy(ctx)


def sf_last_error(ctx):
    return lib().sf_last_error(ctx).decode()


def sf_patch_create(ctx, d, order, knots, ctrl, ctrl_on_device=False):
    """knots: list of d 1D float64 arrays; order: one int for every direction
    or a sequence of d ints; ctrl: host numpy [N, d] or a device tensor."""
    desc = PatchDesc()
    desc.d = d
    orders = [int(order)] * 3 if np.ndim(order) == 0 else [int(o) for o in order] + [0] * (3 - len(order))
    for k in range(3):
        desc.order[k] = orders[k]
    keep = []
    for k in range(3):
        if k < d:
            a = np.ascontiguousarray(knots[k], dtype=np.float64)
            keep.append(a)
            desc.n_knots[k] = len(a)
            desc.knots[k] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            desc.n_knots[k] = 0
    if ctrl_on_device:
        desc.ctrl = _ptr(ctrl)
        desc.ctrl_on_device = 1
    else:
        c = np.ascontiguousarray(ctrl, dtype=np.float64)
        keep.append(c)
        desc.ctrl = c.ctypes.data
        desc.ctrl_on_device = 0
    out = ctypes.c_void_p()
    _check(lib().sf_patch_create(ctx, ctypes.byref(desc), ctypes.byref(out)), ctx)
    return out.value


def sf_patch_info(patch):
    n, z, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = lib().sf_patch_info(patch, ctypes.byref(n), ctypes.byref(z), ctypes.byref(q))
    if st != SF_OK:
        raise SfError(st, "sf_patch_info")
    return n.value, z.value, q.value


def sf_patch_set_coef(ctx, patch, op, kind, value=None, qp_values=None):
    if kind == SF_COEF_QPVALUES:
        arg = ctypes.c_void_p(_ptr(qp_values))
        _check(lib().sf_patch_set_coef(patch, op, kind, arg), ctx)
    else:
        v = (ctypes.c_double * 1)(float(value))
        _check(lib().sf_patch_set_coef(patch, op, kind, ctypes.cast(v, ctypes.c_void_p)), ctx)


def sf_patch_set_convection(ctx, patch, b):
    v = (ctypes.c_double * len(b))(*[float(t) for t in b])
    _check(lib().sf_patch_set_convection(patch, ctypes.cast(v, ctypes.c_void_p)), ctx)


def sf_patch_set_diffusion(ctx, patch, A_upper):
    """A_upper: the d(d+1)/2 upper-triangle entries of the symmetric A, row by row."""
    v = (ctypes.c_double * len(A_upper))(*[float(t) for t in A_upper])
    _check(lib().sf_patch_set_diffusion(patch, ctypes.cast(v, ctypes.c_void_p)), ctx)


def sf_patch_quad_points(ctx, patch, xyz):
    _check(lib().sf_patch_quad_points(patch, _ptr(xyz)), ctx)


def sf_patch_eval(ctx, patch, u, val=None, grad=None):
    _check(lib().sf_patch_eval(patch, _ptr(u), _ptr(val), _ptr(grad)), ctx)


def sf_patch_prepare(ctx, patch, ops, prec=SF_FP64):
    _check(lib().sf_patch_prepare(patch, ops, prec), ctx)


def sf_patch_prepare_async(ctx, patch, ops, prec=SF_FP64):
    _check(lib().sf_patch_prepare_async(patch, ops, prec), ctx)


def sf_patch_geometry_check(ctx, patch):
    _check(lib().sf_patch_geometry_check(patch), ctx)


def sf_csr_pattern(ctx, patch, row_ptr, col_ind):
    _check(lib().sf_csr_pattern(patch, _ptr(row_ptr), _ptr(col_ind)), ctx)


def sf_assemble(ctx, patch, ops, prec, val_mass=None, val_stiff=None):
    _check(lib().sf_assemble(patch, ops, prec, _ptr(val_mass), _ptr(val_stiff)), ctx)


def sf_assemble_noalloc(ctx, patch, ops, prec, val_mass=None, val_stiff=None):
    _check(lib().sf_assemble_noalloc(patch, ops, prec, _ptr(val_mass), _ptr(val_stiff)), ctx)


def sf_apply(ctx, patch, op, prec, x, y):
    _check(lib().sf_apply(patch, op, prec, _ptr(x), _ptr(y)), ctx)


def sf_patch_destroy(patch):
    lib().sf_patch_destroy(patch)


def sf_batch_create(ctx, patches):
    arr = (ctypes.c_void_p * len(patches))(*patches)
    out = ctypes.c_void_p()
    _check(lib().sf_batch_create(ctx, len(patches), arr, ctypes.byref(out)), ctx)
    return out.value


def sf_batch_offsets(ctx, batch, npatch):
    ro = np.zeros(npatch + 1, dtype=np.int64)
    zo = np.zeros(npatch + 1, dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _check(lib().sf_batch_offsets(batch, ro.ctypes.data_as(i64p), zo.ctypes.data_as(i64p)), ctx)
    return ro, zo


def sf_batch_assemble(ctx, batch, ops, prec, row_ptr, col_ind, val_mass=None, val_stiff=None):
    _check(lib().sf_batch_assemble(batch, ops, prec, _ptr(row_ptr), _ptr(col_ind), _ptr(val_mass),
                                   _ptr(val_stiff)), ctx)


def sf_batch_apply(ctx, batch, op, prec, x, y):
    _check(lib().sf_batch_apply(batch, op, prec, _ptr(x), _ptr(y)), ctx)


def sf_glue_map(d, nfuns, interfaces):
    """Host: nfuns [npatch][<=3] functions per direction, interfaces
    [(patch a, face fa, patch b, face fb)]; returns (map int64 [sum N], n_global)."""
    nf = np.zeros((len(nfuns), 3), dtype=np.int32)
    for b, n in enumerate(nfuns):
        nf[b, :len(n)] = n
    ifc = np.ascontiguousarray(np.asarray(interfaces, dtype=np.int32).reshape(-1, 4))
    total = int(sum(np.prod(n[:d]) for n in nfuns))
    m = np.zeros(total, dtype=np.int64)
    ng = ctypes.c_int64()
    st = lib().sf_glue_map(d, len(nfuns), nf.ctypes.data, len(ifc), ifc.ctypes.data if len(ifc) else None,
                           m.ctypes.data, ctypes.byref(ng))
    if st != SF_OK:
        raise SfError(st, "sf_glue_map")
    return m, ng.value


def sf_batch_apply_glued(ctx, batch, op, prec, dev_map, n_global, x, y):
    _check(lib().sf_batch_apply_glued(batch, op, prec, _ptr(dev_map), int(n_global), _ptr(x), _ptr(y)), ctx)


def sf_batch_destroy(batch):
    lib().sf_batch_destroy(batch)
