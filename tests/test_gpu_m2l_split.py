"""The M2L list split (Sec. 5.3 item 3 with each tile's interaction lists
cut into S shares, one block each, the parts added by the downward pass):
every S in {1, 2, 4, 8} against the CPU FP64 oracle at 1e-12, on grid plans
(list rule and a MAC theta), the preconditioner's stages and point clouds;
the splits agree with each other to rounding; the default split gives half
the compute units a block; the tuner keeps one of the four and the solve is unchanged."""
import sys

import numpy as np
import pytest

import oracle as o
from paper_1308_3339_amd import inputs

pytestmark = pytest.mark.gpu

SPLITS = (1, 2, 4, 8)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty(m):
    import torch
    return torch.empty(m, dtype=torch.float64, device="cuda")


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,theta", [(64, None), (256, None), (1024, None), (128, 0.4)])
def test_every_split_matches_oracle(n, theta):
    import paper_1308_3339_amd as fp
    p = 10 if theta is None else 6
    say("case m2l split fmm_apply n=%d p=%d theta=%s" % (n, p, theta))
    q = inputs.random_charges(n * n, seed=3100 + n)
    uo = o.grid_fmm(n, p, q, theta=theta)
    out = {}
    with fp.fmm_setup(n=n, p=p, bem=0, theta=0.0 if theta is None else theta) as plan:
        for split in SPLITS:
            plan.set_m2l_split(split)
            assert plan.m2l_split == split
            u = empty(n * n)
            plan.apply(dev(q), u)
            out[split] = host(u)
            err = relmax(out[split], uo)
            say("  split %d: max rel err vs oracle %.3e" % (split, err))
            assert err <= 1e-12
    for split in SPLITS[1:]:
        assert relmax(out[split], out[1]) <= 1e-14


@pytest.mark.timeout(300)
def test_every_split_preconditioner_stages_match_oracle():
    import paper_1308_3339_amd as fp
    n, p = 128, 10
    say("case m2l split precond stages n=128")
    r = inputs.gaussian_bumps(n, 16, seed=3200)
    zo, phio, sigo = o.Preconditioner(n, p=p).apply(r, stages=True)
    with fp.fmm_setup(n=n, p=p, bem=1) as plan:
        for split in SPLITS:
            plan.set_m2l_split(split)
            z, phi, sig = empty(n * n), empty(4 * n), empty(4 * n)
            plan.precond_stages(dev(r), z, phi, sig)
            e = {"phi_ring": relmax(host(phi), phio), "sigma": relmax(host(sig), sigo),
                 "z": relmax(host(z), zo)}
            say("  split %d:" % split, e)
            assert e["phi_ring"] <= 1e-12
            assert e["sigma"] <= 1e-11
            assert e["z"] <= 1e-11


@pytest.mark.timeout(300)
def test_every_split_on_a_point_cloud():
    import paper_1308_3339_amd as fp
    N, p = 20000, 10
    say("case m2l split points N=20000")
    x, y, q = inputs.random_points(N, seed_xy=3300, seed_q=3301)
    uo = o.fmm(fp.points_levels(N), 0.0, 0.0, 1.0, p, x, y, q, x, y, 0.0)
    with fp.fmm_setup(kind=fp.FMM_POINTS, n=N, p=p, x=dev(x), y=dev(y)) as plan:
        for split in SPLITS:
            plan.set_m2l_split(split)
            u = empty(N)
            plan.apply(dev(q), u)
            err = relmax(host(u), uo)
            say("  split %d: max rel err vs oracle %.3e" % (split, err))
            assert err <= 1e-12


def test_default_split_gives_half_the_units_a_block():
    import torch

    import paper_1308_3339_amd as fp
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    say("case m2l default split, %d compute units" % ncu)
    for n in (64, 256, 1024, 2048):
        L = int(np.log2(n // 8))
        tiles = sum(max(1, ((1 << l) // 16) ** 2) for l in range(2, L + 1))
        split = 1
        while split < 8 and 2 * split * tiles < ncu:
            split *= 2
        with fp.fmm_setup(n=n, p=8, bem=0) as plan:
            say("  n=%d tiles %d default split %d" % (n, tiles, plan.m2l_split))
            assert plan.m2l_split == split


@pytest.mark.timeout(300)
def test_tuned_split_keeps_the_solve():
    import torch

    import paper_1308_3339_amd as fp
    n = 1024
    say("case m2l tuner n=1024")
    f = dev(inputs.gaussian_bumps(n, 16, seed=inputs.SEED_BUMPS_1024))
    with fp.fmm_setup(n=n, p=10) as plan:
        u0 = torch.zeros_like(f)
        i0 = plan.solve(f, u0)
        split = plan.tune_m2l()
        say("  tuned split", split)
        assert split in SPLITS and plan.m2l_split == split
        u1 = torch.zeros_like(f)
        i1 = plan.solve(f, u1)
        assert i1["iters"] == i0["iters"]
        assert relmax(host(u1), host(u0)) <= 1e-10
        assert i1["true_rel_res"] <= 1e-8


def test_split_rejects_bad_values():
    import paper_1308_3339_amd as fp
    say("case m2l split bad values")
    with fp.fmm_setup(n=64, p=8, bem=0) as plan:
        for bad in (0, 3, 16, -1):
            with pytest.raises(fp.FmmError) as ei:
                plan.set_m2l_split(bad)
            assert ei.value.code == fp.FMM_ERR_ARG
        assert plan.m2l_split in SPLITS


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name", ["FMM_SPLIT_FP16", "FMM_SPLIT_BF16"])
def test_matrix_core_m2l_every_split_and_stacked(name):
    """The split 16-bit plans' M2L on the matrix cores: each split against the
    FP64 oracle FMM (the stage bar of the split plans), the splits and a
    stacked three-RHS call against the single calls to FP32 rounding."""
    import paper_1308_3339_amd as fp
    n, p = 256, 10
    bar = 1e-5 if name == "FMM_SPLIT_FP16" else 5e-5
    say("case matrix-core M2L %s n=%d" % (name, n))
    Q = np.stack([inputs.random_charges(n * n, seed=3400 + k) for k in range(3)])
    uo = o.grid_fmm(n, p, Q[0])
    with fp.fmm_setup(n=n, p=p, bem=0, prec=getattr(fp, name)) as plan:
        out = {}
        for split in SPLITS:
            plan.set_m2l_split(split)
            u = empty(n * n)
            plan.apply(dev(Q[0]), u)
            out[split] = host(u)
            err = relmax(out[split], uo)
            say("  split %d: max rel err vs oracle %.3e" % (split, err))
            assert err <= bar
        for split in SPLITS[1:]:
            assert relmax(out[split], out[1]) <= 2e-6
        plan.set_m2l_split(4)
        U = empty(3 * n * n)
        plan.apply(dev(Q.reshape(-1)), U, nrhs=3)
        Ug = host(U).reshape(3, -1)
        for k in range(3):
            u = empty(n * n)
            plan.apply(dev(Q[k]), u)
            d = relmax(Ug[k], host(u))
            say("  stacked rhs %d vs single: %.3e" % (k, d))
            assert d <= 2e-6
