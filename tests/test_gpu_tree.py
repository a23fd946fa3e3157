"""The point-cloud tree built on the device (Sec. 5.1) against the oracle's
bucketing, bit for bit: the permutation (sorted position -> caller index)
and the leaf ranges, leaves in Morton order, points of a leaf in their
original order.  Cases: the 1M-point benchmark cloud, a tight cluster over a
uniform background (one leaf holding most points), every point in one leaf,
points on cell edges and outside the root square (the clamp rule), and the
smallest trees (N = 1, 64, 65).  A non-finite coordinate is rejected."""
import sys

import numpy as np
import pytest

import oracle as o
from paper_1308_3339_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _gpu_order(x, y, x0=0.0, y0=0.0, side=1.0):
    import torch

    import paper_1308_3339_amd as fp
    N = len(x)
    L = fp.points_levels(N)
    with fp.fmm_setup(kind=fp.FMM_POINTS, n=N, p=4, x=dev(x), y=dev(y), x0=x0, y0=y0,
                      side=side) as plan:
        perm = torch.full((N,), -1, dtype=torch.int32, device="cuda")
        start = torch.full(((1 << (2 * L)) + 1,), -1, dtype=torch.int32, device="cuda")
        plan.points_order(perm, start)
        torch.cuda.synchronize()
        return L, perm.cpu().numpy(), start.cpu().numpy()


def _check(x, y, x0=0.0, y0=0.0, side=1.0):
    L, perm, start = _gpu_order(x, y, x0, y0, side)
    so, oo = o.bucket_points(L, x0, y0, side, x, y, morton=True)
    same_start = np.array_equal(start, so)
    same_perm = np.array_equal(perm, oo)
    say("  N=%d L=%d leaf ranges equal %s, permutation equal %s" % (len(x), L, same_start, same_perm))
    assert same_start
    assert same_perm


def test_tree_of_the_benchmark_cloud():
    say("case tree 1M uniform points")
    x, y, _ = inputs.random_points(1 << 20)
    _check(x, y)


def test_tree_of_a_cluster_over_a_background():
    say("case tree clustered 300k points")
    r = np.random.default_rng(91)
    xc = np.clip(r.normal(0.3, 1e-4, 250000), 0.0, 1.0)
    yc = np.clip(r.normal(0.7, 1e-4, 250000), 0.0, 1.0)
    xb, yb, _ = inputs.random_points(50000, seed_xy=92, seed_q=93)
    idx = r.permutation(300000)
    x = np.concatenate([xc, xb])[idx]
    y = np.concatenate([yc, yb])[idx]
    _check(x, y)


def test_tree_with_every_point_in_one_leaf():
    say("case tree one leaf")
    r = np.random.default_rng(94)
    N = 70000              # L = 6: leaves of width 1/64
    w = 1.0 / (1 << 6)
    x = 0.5 + w * r.uniform(0.0, 0.99, N)
    y = 0.25 + w * r.uniform(0.0, 0.99, N)
    _check(x, y)


def test_tree_with_edge_and_outside_points():
    say("case tree edges and outside points")
    r = np.random.default_rng(95)
    N = 5000
    x0, y0, side = -1.0, 2.0, 4.0
    nl = 16   # L = ceil(log4(5000 / 64)) = 4: the points sit on leaf edges
    k = r.integers(0, nl + 1, N)
    j = r.integers(0, nl + 1, N)
    x = x0 + side * k / nl
    y = y0 + side * j / nl
    # some outside the root square, some duplicated points
    x[:200] = x0 - r.uniform(0.0, 3.0, 200)
    y[200:400] = y0 + side + r.uniform(0.0, 3.0, 200)
    x[400:600] = x[600:800]
    y[400:600] = y[600:800]
    _check(x, y, x0, y0, side)


@pytest.mark.parametrize("N", [1, 64, 65, 4097])
def test_tree_of_small_clouds(N):
    say("case tree N=%d" % N)
    x, y, _ = inputs.random_points(N, seed_xy=96 + N, seed_q=97)
    _check(x, y)


def test_tree_rejects_non_finite_coordinates():
    import paper_1308_3339_amd as fp
    say("case tree NaN coordinate")
    x, y, _ = inputs.random_points(1000, seed_xy=98, seed_q=99)
    x[517] = np.nan
    with pytest.raises(fp.FmmError) as ei:
        fp.fmm_setup(kind=fp.FMM_POINTS, n=1000, p=4, x=dev(x), y=dev(y))
    assert ei.value.code == fp.FMM_ERR_ARG
