"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the
oracle.  This module holds no part of the method's arithmetic: it only builds
knot vectors, control points and vectors that both sides take as input.

Recipe (the paper's own test geometries, a quarter annulus and a bent and
twisted box, are not given in a reproducible form, so these stand in):

* knots: open, uniform, interior multiplicity one, on [0, 1];
* geometry: control points at the Greville abscissae of the tensor-product
  basis (the identity map, by linear precision), then every component of
  every control point moved by ``U(-0.05, 0.05) * h_delta`` with
  ``h_delta = 1 / K_delta`` (NumPy ``default_rng``, PCG64);
* vectors: ``x ~ U(-1, 1)``;
* batched sets: ``K_delta ~ U{4..32}``, ``p ~ U{2..6}``, patch ``b`` uses
  geometry seed ``[1, b]`` and vector seed ``[0, b]``.
"""
from __future__ import annotations

import numpy as np


def open_uniform_knots(K: int, p: int) -> np.ndarray:
    """Open uniform knot vector of order p (degree p-1) with K elements."""
    inner = np.arange(1, K, dtype=np.float64) / K
    return np.concatenate([np.zeros(p), inner, np.ones(p)])


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae xi_i = (t_{i+1} + ... + t_{i+p-1}) / (p-1), order p >= 2."""
    t = np.asarray(knots, dtype=np.float64)
    n = len(t) - p
    if p < 2:
        raise ValueError("Greville abscissae need order >= 2")
    return np.array([t[i + 1:i + p].sum() / (p - 1) for i in range(n)])


def greville_grid(knots_list, orders) -> np.ndarray:
    """Control points [N, d] at the tensor Greville points, lexicographic with
    direction 1 fastest."""
    axes = [greville(k, p) for k, p in zip(knots_list, orders)]
    mesh = np.meshgrid(*axes, indexing="ij")          # mesh[i][j1, j2, ...]
    d = len(axes)
    # flatten with direction 1 fastest: transpose so that axis 0 varies fastest
    cols = [m.transpose(*range(d - 1, -1, -1)).reshape(-1) for m in mesh]
    return np.stack(cols, axis=1)


def perturbed_geometry(K, p, seed=1, amp=0.05, interior_only=False):
    """Knots and control points of the perturbed-Greville patch."""
    d = len(K)
    knots = [open_uniform_knots(k, p) for k in K]
    ctrl = greville_grid(knots, [p] * d)
    rng = np.random.default_rng(seed)
    h = np.array([1.0 / k for k in K])
    delta = rng.uniform(-amp, amp, size=ctrl.shape) * h[None, :]
    if interior_only:
        nf = [k + p - 1 for k in K]
        idx = np.indices(nf[::-1]).reshape(d, -1)[::-1]     # per-direction index, dir 1 fastest
        inner = np.ones(ctrl.shape[0], dtype=bool)
        for k in range(d):
            inner &= (idx[k] > 0) & (idx[k] < nf[k] - 1)
        delta[~inner] = 0.0
    return knots, ctrl + delta


def identity_geometry(K, p):
    d = len(K)
    knots = [open_uniform_knots(k, p) for k in K]
    return knots, greville_grid(knots, [p] * d)


def random_vector(n: int, seed=0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def ndof(K, p) -> int:
    return int(np.prod([k + p - 1 for k in K]))


# ------------------------------------------------------------ workloads

def workload_small_2d():
    """d=2, 16x16 elements, order 3, identity geometry, a = c = 1."""
    K, p = (16, 16), 3
    knots, ctrl = identity_geometry(K, p)
    return dict(name="d2_16x16_p3_identity", K=K, p=p, knots=knots, ctrl=ctrl,
                coef=("const", 1.0), x=random_vector(ndof(K, p), 0))


def workload_3d(K=(48, 48, 48), p=4, alpha=0.5):
    """d=3 perturbed-Greville patch with a(x) = 1 + alpha sin sin sin."""
    knots, ctrl = perturbed_geometry(K, p, seed=1)
    return dict(name=f"d3_{K[0]}x{K[1]}x{K[2]}_p{p}_perturbed", K=K, p=p, knots=knots,
                ctrl=ctrl, coef=("sinprod", alpha), x=random_vector(ndof(K, p), 0))


def workload_order_sweep(p):
    """d=3, K = 127 - p per direction so that N = 126^3 for every order."""
    K = (127 - p,) * 3
    return workload_3d(K, p)


def batched_draw(npatch=512, seed=2, kmin=4, kmax=32, pmin=2, pmax=6):
    """Per-patch element counts and orders of the batched workload."""
    r = np.random.default_rng(seed)
    K = r.integers(kmin, kmax + 1, size=(npatch, 3))
    p = r.integers(pmin, pmax + 1, size=npatch)
    return K, p


def batched_patch(b, K, p):
    knots = [open_uniform_knots(int(k), int(p)) for k in K]
    ctrl = greville_grid(knots, [int(p)] * len(K))
    rng = np.random.default_rng([1, b])
    h = np.array([1.0 / k for k in K])
    ctrl = ctrl + rng.uniform(-0.05, 0.05, size=ctrl.shape) * h[None, :]
    x = np.random.default_rng([0, b]).uniform(-1.0, 1.0, ctrl.shape[0])
    return knots, ctrl, x
