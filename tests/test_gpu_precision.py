"""Precision variants against the FP64 oracle: FMM_FP32 (P2P and P2M as FP32
matrix-core contractions, M2L in FP32), FMM_SPLIT_FP16 and FMM_SPLIT_BF16
(P2P and P2M as 16-bit hi+lo products on the matrix cores, M2L in FP32);
everything else FP64.

The variant changes the preconditioner only by rounding, so:
  * per-stage error against the FP64 oracle (volume potential, ring
    potential, z) <= 1e-5 relative (max-norm) for FP32 and
    split FP16; the FP32 sums are 64-term partials folded into FP64, the FMM
    truncation at p = 10 is ~1e-6, so a few 1e-6 is the expected level.
    Split BF16 represents each operand to 2^-16 (1.5e-5) relative, so a
    product carries up to 2^-15; the bar is 5e-5, a little above that per
    product error (the near field's terms are mostly of one sign: the log
    kernel is negative over the whole near field, so sums cancel little);
  * the boundary density is the FP64 solve of the first-kind collocation
    system with the plan's own ring potential, so its error is the ring
    potential's error carried through S^{-1} (amplified up to kappa(S)); the
    test reproduces that propagated error with the oracle's factors of S and
    requires the density to equal it within 1e-9;
  * the flexible outer iteration still reaches the FP64 true residual
    <= 1e-8, within two iterations of the FP64 preconditioner, and the
    solution agrees with the oracle's within 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle as o
from paper_1308_3339_amd import inputs

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


PRECS = ("FMM_FP32", "FMM_SPLIT_FP16", "FMM_SPLIT_BF16")
STAGE_BAR = {"FMM_FP32": 1e-5, "FMM_SPLIT_FP16": 1e-5, "FMM_SPLIT_BF16": 5e-5}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [32, 128, 256])
def test_fp32_stages_against_fp64_oracle(n, prec):
    import torch

    import paper_1308_3339_amd as fp
    say("case %s stages n=%d" % (prec, n))
    p = 10
    r = inputs.random_charges(n * n, seed=600 + n)
    with fp.fmm_setup(n=n, p=p, bem=1, prec=getattr(fp, prec)) as plan:
        u = torch.empty(n * n, dtype=torch.float64, device="cuda")
        plan.apply(dev(r), u)
        z, phi, sig = (torch.empty(m, dtype=torch.float64, device="cuda") for m in (n * n, 4 * n, 4 * n))
        plan.precond_stages(dev(r), z, phi, sig)
        ug, zg, phig, sigg = host(u), host(z), host(phi), host(sig)
    uo = o.grid_fmm(n, p, r)
    pc = o.Preconditioner(n, p=p)
    zo, phio, sigo = pc.apply(r, stages=True)
    errs = {"volume": relmax(ug, uo), "phi_ring": relmax(phig, phio), "sigma": relmax(sigg, sigo),
            "z": relmax(zg, zo)}
    # sigma is the FP64 boundary solve of the plan's own ring potential: its
    # error is the ring potential's carried through S^{-1} (Sec. 4.3), which
    # the oracle's own factors of S reproduce
    errs["sigma_vs_propagated"] = relmax(sigg, sigo + pc.bem_solve(phig - phio))
    say("  per-stage rel err vs FP64 oracle", errs)
    for k in ("volume", "phi_ring", "z"):
        assert errs[k] <= STAGE_BAR[prec], k
    assert errs["sigma_vs_propagated"] <= 1e-9


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [64, 256])
def test_fp32_solve_reaches_fp64_residual(n, prec):
    import torch

    import paper_1308_3339_amd as fp
    say("case %s solve n=%d" % (prec, n))
    f = inputs.gaussian_bumps(n, 16, seed=700 + n)
    its = {}
    sols = {}
    low = getattr(fp, prec)
    for prec in (fp.FMM_FP64, low):
        with fp.fmm_setup(n=n, p=10, prec=prec) as plan:
            u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
            info = plan.solve(dev(f), u)
            assert info["converged"]
            sols[prec], its[prec] = host(u), info["iters"]
    say("  iterations fp64 %d reduced %d" % (its[fp.FMM_FP64], its[low]))
    res = np.linalg.norm(f - o.stencil(n, sols[low])) / np.linalg.norm(f)
    assert res <= 1e-8
    assert its[low] <= its[fp.FMM_FP64] + 2
    xo, _ = o.fgmres(n, f, o.Preconditioner(n, p=10))
    assert np.linalg.norm(sols[low] - xo) <= 1e-6 * np.linalg.norm(xo)


@pytest.mark.parametrize("prec", PRECS)
def test_fp32_full_size_solve(prec):
    import torch

    import paper_1308_3339_amd as fp
    n = 2048
    say("case %s solve n=2048" % prec)
    f = inputs.gaussian_bumps(n, 16, seed=inputs.SEED_BUMPS_2048)
    with fp.fmm_setup(n=n, p=10, prec=getattr(fp, prec)) as plan:
        u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
        info = plan.solve(dev(f), u)
        ug = host(u)
    say("  info", info)
    assert info["converged"]
    res = np.linalg.norm(f - o.stencil(n, ug)) / np.linalg.norm(f)
    say("  CPU-recomputed true rel res %.3e" % res)
    assert res <= 1e-8


@pytest.mark.parametrize("prec", ["FMM_SPLIT_FP16", "FMM_SPLIT_BF16"])
def test_split_leaf_tile_loop_stacked(prec):
    """The split 16-bit leaf kernel runs two blocks per compute unit over all
    right-hand sides, each block looping over 8 x 8-leaf tiles with the next
    tile's charges loaded during the current one's products.  A stacked call
    of 8 right-hand sides at 1024^2 (256 tiles each, 64 blocks per right-hand
    side: 4 tiles per block) against single calls (one tile per block): the
    near field and P2M are computed tile by tile in the same order either way,
    and the stacked call's M2L takes a smaller list split, so the
    applications agree to the M2L parts' rounding; a tile or right-hand side
    mixed up in the loop would differ at O(1)."""
    import torch

    import paper_1308_3339_amd as fp
    n, nr = 1024, 8
    say("case %s stacked leaf tile loop n=%d nrhs=%d" % (prec, n, nr))
    Q = np.stack([inputs.random_charges(n * n, seed=4100 + k) for k in range(nr)])
    with fp.fmm_setup(n=n, p=10, bem=0, prec=getattr(fp, prec)) as plan:
        U = torch.empty(nr * n * n, dtype=torch.float64, device="cuda")
        plan.apply(dev(Q.reshape(-1)), U, nrhs=nr)
        Ug = host(U).reshape(nr, -1)
        for k in range(nr):
            u = torch.empty(n * n, dtype=torch.float64, device="cuda")
            plan.apply(dev(Q[k]), u)
            d = relmax(Ug[k], host(u))
            say("  rhs %d stacked vs single: %.3e" % (k, d))
            assert d <= 2e-6
