"""Pins of the oracle's glued multipatch operator (Sec. 4, Example
"Multipatch domains"): sum_b R_b^T A_b R_b over conforming patches whose
interface functions are identified.

The pin is a fact about splines, not the oracle: a single patch whose knot
vector repeats an interior knot p - 1 times (C0 there) has a basis that is
exactly the glued basis of the two patches on either side (each with an
open knot vector, rescaled to [0, 1]); with the same control points the
geometry, the quadrature elements and so every matrix agree.  The oracle
assembles the C0 patch directly (it takes interior knots of multiplicity up
to p) and the glued one from the pieces."""
import numpy as np
import pytest

import oracle
from paper_1809_05471_amd import inputs


def c0_split(K, splits, p, seed, amp=0.08):
    """A C0 patch and its glued pieces.  K: elements per direction; splits:
    per direction the element counts of the pieces (summing to K).  Returns
    (knots, ctrl of the C0 patch, pieces), pieces = list of (knots, ctrl,
    nfun, index of each piece function in the C0 patch)."""
    d = len(K)
    kn0, offs1, nf0 = [], [], []
    for k in range(d):
        br = np.linspace(0.0, 1.0, K[k] + 1)
        inner = []
        cuts = np.cumsum(splits[k])[:-1]
        for e in range(1, K[k]):
            inner += [br[e]] * ((p - 1) if e in cuts else 1)
        kn0.append(np.concatenate([np.zeros(p), inner, np.ones(p)]))
        nf0.append(len(kn0[-1]) - p)
        # first C0 function of each piece: pieces share their end function
        firsts, f = [], 0
        for ne in splits[k]:
            firsts.append(f)
            f += ne + p - 2
        offs1.append(firsts)
    ctrl0 = inputs.greville_grid(kn0, [p] * d)
    rng = np.random.default_rng(seed)
    h = np.array([1.0 / k for k in K])
    ctrl0 = ctrl0 + rng.uniform(-amp, amp, size=ctrl0.shape) * h[None, :] / p
    pieces = []
    for pidx in np.ndindex(*[len(s) for s in splits]):
        kn, nf, idx1 = [], [], []
        for k in range(d):
            kn.append(inputs.open_uniform_knots(splits[k][pidx[k]], p))
            nf.append(splits[k][pidx[k]] + p - 1)
            idx1.append(offs1[k][pidx[k]] + np.arange(nf[-1]))
        # lexicographic, direction 1 fastest
        grids = np.meshgrid(*idx1[::-1], indexing="ij")
        lin = np.zeros(grids[0].shape, dtype=np.int64)
        stride = 1
        for k in range(d):
            lin += grids[d - 1 - k] * stride
            stride *= nf0[k]
        c0_index = lin.ravel()
        pieces.append((kn, ctrl0[c0_index], nf, c0_index))
    return kn0, ctrl0, pieces


def interfaces_of(splits):
    """Faces shared by neighbouring pieces of the grid of pieces."""
    d = len(splits)
    shape = [len(s) for s in splits]
    ids = {pidx: i for i, pidx in enumerate(np.ndindex(*shape))}
    out = []
    for pidx, i in ids.items():
        for k in range(d):
            q = list(pidx)
            q[k] += 1
            if q[k] < shape[k]:
                out.append((i, 2 * k + 1, ids[tuple(q)], 2 * k))
    return out


CASES = [((6,), ((2, 4),), 3), ((5, 4), ((2, 3), (4,)), 2), ((4, 5), ((2, 2), (3, 2)), 3),
         ((4, 3, 2), ((2, 2), (1, 2), (2,)), 2), ((3, 4, 2), ((1, 2), (2, 2), (1, 1)), 3)]


@pytest.mark.parametrize("K,splits,p", CASES)
def test_c0_patch_equals_glued_pieces(K, splits, p):
    d = len(K)
    kn0, ctrl0, pieces = c0_split(K, splits, p, seed=7)
    single = oracle.Problem(kn0, p, ctrl0, ("sinprod", 0.4), conv_b=(0.5, -0.7, 0.3)[:d])
    maps, ng = oracle.glue_map(d, [pc[2] for pc in pieces], interfaces_of(splits))
    assert ng == single.N
    probs = [oracle.Problem(kn, p, c, ("sinprod", 0.4), conv_b=(0.5, -0.7, 0.3)[:d]) for kn, c, _, _ in pieces]
    # the glued numbering is a relabelling of the C0 patch's functions
    perm = np.full(ng, -1)
    for m, (_, _, _, c0i) in zip(maps, pieces):
        assert np.all((perm[m] == -1) | (perm[m] == c0i))
        perm[m] = c0i
    assert sorted(perm.tolist()) == list(range(single.N))
    ops = [oracle.MASS, oracle.STIFF] + ([oracle.CONV] if d >= 2 else [])
    for op in ops:
        A0 = single.dense(op)
        G = oracle.glued_dense(probs, maps, ng, op)
        assert np.abs(G - A0[np.ix_(perm, perm)]).max() <= 1e-13 * np.abs(A0).max()
        x = inputs.random_vector(ng, 3)
        y = oracle.glued_apply(probs, maps, ng, op, x)
        assert np.abs(y - G @ x).max() <= 1e-13 * np.abs(G).max() * np.abs(x).max() * 10


def test_glue_map_counts_and_refusal():
    # 2 x 2 pieces in 2D of 4 x 5 functions each: 2 shared lines of 5 and 4,
    # the centre function in all four
    nf = [[4, 5], [4, 5], [4, 5], [4, 5]]
    maps, ng = oracle.glue_map(2, nf, [(0, 1, 1, 0), (2, 1, 3, 0), (0, 3, 2, 2), (1, 3, 3, 2)])
    assert ng == 4 * 20 - 2 * 5 - 2 * 4 + 1
    assert len(set(np.concatenate(maps).tolist())) == ng
    with pytest.raises(oracle.OracleError):
        oracle.glue_map(2, [[4, 5], [4, 6]], [(0, 1, 1, 0)])
