"""FMM_FP32 point-cloud plans: the near field pairwise in FP32 with the
polynomial logarithm and Kahan-compensated sums (Secs. 5.3, 7.1), the far
field FP64, through the C ABI.

Bar: within 1e-5 (max-norm, relative to max |u|) of the oracle's FP64 FMM at
the same p, the bar of the other reduced-precision stages.  The arithmetic
gives far less: each pair carries about 1e-7 relative error (FP32 offsets,
charges and logarithm), and compensated sums keep the ~600 near pairs of a
target from accumulating more than that per term.  The FP32 result must also
differ from the FP64 plan's (the FP32 kernel ran), and reach the direct sum
as closely as the FP64 FMM does at p = 12.
"""
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


def run(x, y, q, p, prec, theta=0.0):
    import torch

    import paper_1308_3339_amd as fp
    N = len(x)
    with fp.fmm_setup(kind=fp.FMM_POINTS, n=N, p=p, x=dev(x), y=dev(y), prec=prec,
                      theta=theta) as plan:
        u = torch.empty(N, dtype=torch.float64, device="cuda")
        plan.apply(dev(q), u)
        torch.cuda.synchronize()
        return u.cpu().numpy()


def levels(N):
    L = 0
    while (64 << (2 * L)) < N:
        L += 1
    return L


def test_points_fp32_single_point():
    import paper_1308_3339_amd as fp
    x, y, q = np.array([0.3]), np.array([0.7]), np.array([1.5])
    assert np.array_equal(run(x, y, q, 6, fp.FMM_FP32), np.zeros(1))


def test_points_fp32_with_list_rule_theta():
    """theta = 0.8 > 1/sqrt(2) gives the list rule's lists (the only theta FP32
    plans take): the same result as theta = 0 bit for bit."""
    import paper_1308_3339_amd as fp
    N, p = 5000, 8
    x, y, q = inputs.random_points(N, seed_xy=1401, seed_q=1402)
    assert np.array_equal(run(x, y, q, p, fp.FMM_FP32, theta=0.8), run(x, y, q, p, fp.FMM_FP32))


@pytest.mark.parametrize("N,p", [(2, 6), (300, 8), (5000, 10), (20000, 10), (100000, 10)])
def test_points_fp32_match_oracle(N, p):
    import paper_1308_3339_amd as fp
    say("case points fp32 N=%d p=%d" % (N, p))
    x, y, q = inputs.random_points(N, seed_xy=1100 + N, seed_q=1200 + N)
    u32 = run(x, y, q, p, fp.FMM_FP32)
    u64 = run(x, y, q, p, fp.FMM_FP64)
    if N <= 20000:
        uo = o.fmm(levels(N), 0.0, 0.0, 1.0, p, x, y, q, x, y, 0.0)
    else:
        uo = u64     # the FP64 plan matches the oracle to 1e-12 (test_gpu_points.py)
    scale = np.abs(uo).max()
    e32 = np.abs(u32 - uo).max() / scale
    e64 = np.abs(u64 - uo).max() / scale
    say("  max rel err: fp32 %.3e, fp64 %.3e" % (e32, e64))
    assert e32 <= 1e-5
    assert e64 <= 1e-12
    if N > 2:
        assert e32 > e64     # the FP32 kernel is the one that ran


def test_points_fp32_accuracy_against_direct_sum():
    import paper_1308_3339_amd as fp
    N, p = 8192, 12
    say("case points fp32 vs direct N=%d p=%d" % (N, p))
    x, y, q = inputs.random_points(N, seed_xy=1301, seed_q=1302)
    ud = o.direct(x, y, q, x, y, 0.0)
    e = {}
    for prec in (fp.FMM_FP32, fp.FMM_FP64):
        u = run(x, y, q, p, prec)
        e[prec] = np.linalg.norm(u - ud) / np.linalg.norm(ud)
    say("  rel L2 vs direct: fp32 %.3e, fp64 %.3e" % (e[fp.FMM_FP32], e[fp.FMM_FP64]))
    assert e[fp.FMM_FP64] <= 1e-6
    assert e[fp.FMM_FP32] <= 2e-6


def test_points_split_fp16_rejected():
    import paper_1308_3339_amd as fp
    x, y, _ = inputs.random_points(100, seed_xy=1, seed_q=2)
    with pytest.raises(fp.FmmError):
        fp.fmm_setup(kind=fp.FMM_POINTS, n=100, p=6, x=dev(x), y=dev(y), prec=fp.FMM_SPLIT_FP16)


def test_points_fp32_one_million_against_direct_subset():
    """The bare-FMM workload at full size: 1M U(0,1)^2 points, U(-1,1)
    charges, p = 12, FP32 near field, against the direct sum on the seeded
    4096-target subset (the FP64 plan's bar, 1e-6: FP32 adds about 1e-7)."""
    import paper_1308_3339_amd as fp
    say("case points fp32 N=1M p=12")
    N = 1 << 20
    x, y, q = inputs.random_points(N)
    ug = run(x, y, q, 12, fp.FMM_FP32)
    idx = inputs.target_subset(N, 4096)
    ud = o.direct(x, y, q, x[idx], y[idx], 0.0)
    err = np.linalg.norm(ug[idx] - ud) / np.linalg.norm(ud)
    say("  rel L2 vs direct on 4096 targets %.3e" % err)
    assert err <= 1e-6
