"""Pins of the oracle's point bucketing (tree construction of Sec. 5.1 on the
uniform quadtree): leaf keys, the Morton order, the stable counting sort.

Each check is against something the oracle does not compute itself:
  * Morton indices of hand-picked leaves (bit interleaving written out),
  * the parent relation of the quadtree (key at level L >> 2 = key at L - 1)
    and the contiguity of every subtree in the sorted order,
  * numpy's stable argsort of the same keys (a library sort, not a
    counting sort), and np.bincount for the leaf counts,
  * leaves of points placed on cell edges and outside the root square,
    whose leaf follows from the clamp rule by hand.
"""
import numpy as np
import pytest

import oracle as o
from paper_1308_3339_amd import inputs


def _spread_bits(v):
    # 16-bit value with a zero bit inserted above every bit (mask form)
    v = v.astype(np.uint64) & np.uint64(0xFFFF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
    v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
    v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
    v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
    return v


def _morton_np(lx, ly):
    return (_spread_bits(np.asarray(lx)) | (_spread_bits(np.asarray(ly)) << np.uint64(1))).astype(np.int64)


def _leaf_of(x, nl):
    return np.minimum(np.maximum(np.floor(x * nl), 0), nl - 1).astype(np.int64)


def test_morton_indices_of_known_leaves():
    L = 3
    nl = 1 << L
    # one point at the centre of each listed leaf
    cases = {(0, 0): 0, (1, 0): 1, (0, 1): 2, (1, 1): 3, (2, 0): 4, (0, 2): 8, (3, 3): 15,
             (4, 0): 16, (0, 4): 32, (5, 6): 57, (7, 7): 63}
    for (lx, ly), m in cases.items():
        x = np.array([(lx + 0.5) / nl])
        y = np.array([(ly + 0.5) / nl])
        start, order = o.bucket_points(L, 0.0, 0.0, 1.0, x, y, morton=True)
        counts = np.diff(start)
        assert counts[m] == 1 and counts.sum() == 1, (lx, ly)


@pytest.mark.parametrize("L", [1, 4, 7])
def test_bucketing_equals_stable_argsort_of_morton_keys(L):
    N = 20000
    x, y, _ = inputs.random_points(N, seed_xy=40 + L, seed_q=41)
    nl = 1 << L
    keys = _morton_np(_leaf_of(x, nl), _leaf_of(y, nl))
    start, order = o.bucket_points(L, 0.0, 0.0, 1.0, x, y, morton=True)
    assert np.array_equal(order, np.argsort(keys, kind="stable"))
    assert np.array_equal(np.diff(start), np.bincount(keys, minlength=nl * nl))
    assert start[0] == 0 and start[-1] == N


def test_row_major_bucketing_equals_stable_argsort():
    L, N = 5, 5000
    x, y, _ = inputs.random_points(N, seed_xy=50, seed_q=51)
    nl = 1 << L
    keys = _leaf_of(y, nl) * nl + _leaf_of(x, nl)
    start, order = o.bucket_points(L, 0.0, 0.0, 1.0, x, y, morton=False)
    assert np.array_equal(order, np.argsort(keys, kind="stable"))


def test_every_subtree_is_contiguous_and_parents_nest():
    L, N = 6, 30000
    x, y, _ = inputs.random_points(N, seed_xy=60, seed_q=61)
    start, order = o.bucket_points(L, 0.0, 0.0, 1.0, x, y, morton=True)
    xs, ys = x[order], y[order]
    for lev in range(1, L + 1):
        nc = 1 << lev
        cell = _leaf_of(ys, nc) * nc + _leaf_of(xs, nc)
        # contiguous: each cell id appears in one run of the sorted sequence
        runs = cell[np.r_[True, cell[1:] != cell[:-1]]]
        assert len(runs) == len(np.unique(cell)), lev
    # the key of a leaf's parent is the leaf key shifted by two bits
    startp, orderp = o.bucket_points(L - 1, 0.0, 0.0, 1.0, x, y, morton=True)
    cnt = np.diff(start).reshape(-1, 4).sum(axis=1)
    assert np.array_equal(cnt, np.diff(startp))
    # and the leaf segments of one parent, taken together, hold exactly the
    # parent's segment at level L - 1
    for par in range(0, len(cnt), 97):
        a = np.sort(order[start[4 * par]:start[4 * par + 4]])
        b = np.sort(orderp[startp[par]:startp[par + 1]])
        assert np.array_equal(a, b)


def test_edges_and_outside_points_follow_the_clamp_rule():
    L = 3
    nl = 1 << L
    side, x0, y0 = 2.0, -1.0, 0.5
    w = side / nl
    # on cell edges (exactly representable), on the far edge, and outside
    pts = [(x0 + 3 * w, y0 + 0.5 * w, (3, 0)),
           (x0 + 0.5 * w, y0 + 5 * w, (0, 5)),
           (x0 + side, y0 + side, (7, 7)),
           (x0 - 0.25, y0 + 2.5 * w, (0, 2)),
           (x0 + side + 3.0, y0 - 1.0, (7, 0)),
           (x0, y0, (0, 0))]
    x = np.array([p[0] for p in pts])
    y = np.array([p[1] for p in pts])
    start, order = o.bucket_points(L, x0, y0, side, x, y, morton=True)
    counts = np.diff(start)
    for i, (_, _, (lx, ly)) in enumerate(pts):
        m = int(_morton_np(np.array([lx]), np.array([ly]))[0])
        pos = int(np.nonzero(order == i)[0][0])
        assert start[m] <= pos < start[m + 1], (i, lx, ly)
    assert counts.sum() == len(pts)


def test_ties_keep_the_original_order():
    # many points in one leaf and a few elsewhere: the leaf's segment lists
    # them by increasing original index
    L = 2
    x = np.array([0.1, 0.9, 0.1, 0.12, 0.6, 0.11, 0.1])
    y = np.array([0.1, 0.9, 0.1, 0.13, 0.1, 0.14, 0.1])
    start, order = o.bucket_points(L, 0.0, 0.0, 1.0, x, y, morton=True)
    seg = order[start[0]:start[1]]
    assert list(seg) == [0, 2, 3, 5, 6]
