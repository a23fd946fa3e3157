"""The work counts bench.py prices its rooflines with, pinned to the oracle's
own interaction lists (host only, no GPU).

* M2L translations of the list rule (Sec. 5.2, children of the parent's 3x3
  neighbourhood minus the own 3x3 block) in closed form, against the number
  of M2L pairs the oracle's dual tree traversal emits for a theta that
  reproduces that rule (theta = 0.8 > 1/sqrt(2)).
* Near-field pairs of the leaf kernel, 64 x 64 points per P2P leaf pair,
  against the traversal's P2P leaf pairs.
"""
import pytest

import bench
import oracle as o


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_m2l_translation_count_matches_oracle_lists(L):
    m2l, _ = o.dtt_lists(L, 0.8)
    assert len(m2l) == bench.m2l_translations(L)


def test_m2l_translation_count_at_2048():
    # 2048^2 grid: L = 8 (256 x 256 leaves of 8 x 8 points)
    assert bench.m2l_translations(8) == 2316900


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
def test_leaf_pair_count_matches_oracle_lists(L):
    _, p2p = o.dtt_lists(L, 0.8)
    n, p = 8 << L, 10
    near_flops = bench.leaf_kernel_flops(n, p) - 4.0 * p * n * n
    assert near_flops == 2.0 * 64 * 64 * len(p2p)


def test_kernel_source_hashes_find_their_kernels():
    # the committed counter summaries are tied to these hashes: each lookup
    # must find its kernel's declaration in the current sources
    h = bench.leaf_kernel_hash()
    assert len(h) == 64
    for fname, head in bench.POINTS_HEADS.values():
        assert len(bench.kernel_source_hash(fname, head)) == 64
