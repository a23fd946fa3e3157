"""FP32 grid plans with a MAC theta (Sec. 5.2 near disk and lists, Sec. 7.1
single-precision near field): the leaf kernel contracts the disk's leaf
offsets on the FP32 matrix cores, M2L runs in FP32 over the traversal's
lists, everything else stays FP64.  Through the C ABI against the oracle's
FP64 traversal FMM and preconditioner.

Bar: 1e-5 relative (max-norm) for the volume potential, the ring potential
phi_ring and the preconditioner's output z, the bar of the other reduced-
precision plans.  The boundary density sigma solves the first-kind system
S sigma = -phi_ring, which can amplify a relative error of phi_ring by up to
the condition number of S, so sigma's bar is kappa_inf(S) times phi_ring's
measured error (kappa_inf(S) = 450 at 256^2, from the oracle's S).  The
solve reaches the FP64 residual 1e-8 (recomputed on the CPU) in at most one
iteration more than the FP64 plan with the same theta.
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


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty(n):
    import torch
    return torch.empty(n, dtype=torch.float64, device="cuda")


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,p,theta", [(32, 6, 0.4), (64, 6, 0.4), (128, 6, 0.4), (256, 6, 0.4),
                                       (128, 8, 0.55), (256, 6, 0.3), (64, 10, 0.55)])
def test_fp32_theta_fmm_apply_matches_oracle(n, p, theta):
    import paper_1308_3339_amd as fp
    say("case fp32 theta fmm_apply n=%d p=%d theta=%g" % (n, p, theta))
    q = inputs.random_charges(n * n, seed=1500 + n + p)
    out = {}
    for prec in (fp.FMM_FP32, fp.FMM_FP64):
        with fp.fmm_setup(n=n, p=p, bem=0, theta=theta, prec=prec) as plan:
            u = empty(n * n)
            plan.apply(dev(q), u)
            out[prec] = host(u)
    uo = o.grid_fmm(n, p, q, theta=theta)
    e32, e64 = relmax(out[fp.FMM_FP32], uo), relmax(out[fp.FMM_FP64], uo)
    say("  max rel err vs oracle: fp32 %.3e, fp64 %.3e" % (e32, e64))
    assert e32 <= 1e-5
    assert e64 <= 1e-12
    assert e32 > e64


@pytest.mark.parametrize("n,p,theta", [(64, 6, 0.4), (256, 6, 0.4), (128, 8, 0.3)])
def test_fp32_theta_precond_stages_match_oracle(n, p, theta):
    import paper_1308_3339_amd as fp
    say("case fp32 theta precond stages n=%d p=%d theta=%g" % (n, p, theta))
    r = inputs.random_charges(n * n, seed=1600 + n)
    with fp.fmm_setup(n=n, p=p, bem=1, theta=theta, prec=fp.FMM_FP32) as plan:
        z, phi, sig = empty(n * n), empty(4 * n), empty(4 * n)
        plan.precond_stages(dev(r), z, phi, sig)
        zg, phig, sigg = host(z), host(phi), host(sig)
    zo, phio, sigo = o.Preconditioner(n, p=p, theta=theta).apply(r, stages=True)
    e_phi, e_sig, e_z = relmax(phig, phio), relmax(sigg, sigo), relmax(zg, zo)
    kappa = float(np.linalg.cond(o.bem_matrix(n), np.inf))
    say("  phi_ring %.2e sigma %.2e z %.2e, kappa_inf(S) %.1f" % (e_phi, e_sig, e_z, kappa))
    assert e_phi <= 1e-5 and e_z <= 1e-5
    assert e_sig <= kappa * e_phi


@pytest.mark.parametrize("n", [256, 2048])
def test_fp32_theta_solve(n):
    import torch

    import paper_1308_3339_amd as fp
    say("case fp32 theta solve n=%d" % n)
    seed = inputs.SEED_BUMPS_2048 if n == 2048 else 1700 + n
    f = inputs.gaussian_bumps(n, 16, seed=seed)
    its = {}
    for prec in (fp.FMM_FP32, fp.FMM_FP64):
        with fp.fmm_setup(n=n, p=6, theta=0.4, prec=prec) as plan:
            u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
            info = plan.solve(dev(f), u)
            ug = host(u)
        say("  prec %d info %s" % (prec, info))
        assert info["converged"]
        its[prec] = info["iters"]
        res = np.linalg.norm(f - o.stencil(n, ug)) / np.linalg.norm(f)
        say("  CPU-recomputed true rel res %.3e" % res)
        assert res <= 1e-8
    assert its[fp.FMM_FP32] <= its[fp.FMM_FP64] + 1


def test_fp32_theta_fullsize_sampled_against_direct():
    """2048^2, p = 6, theta = 0.4 (the configuration bench.py times) with the
    FP32 near field and M2L: 512 sampled nodes against the direct sum, within
    the FP64 theta plan's bar (2e-6: truncation about 1e-6, FP32 adds about
    2e-7)."""
    import paper_1308_3339_amd as fp
    n = 2048
    say("case fp32 theta fullsize sampled")
    q = inputs.random_charges(n * n, seed=77)
    with fp.fmm_setup(n=n, p=6, bem=0, theta=0.4, prec=fp.FMM_FP32) as plan:
        u = empty(n * n)
        plan.apply(dev(q), u)
        ug = host(u)
    idx = inputs.target_subset(n * n, 512, seed=78)
    gx, gy = o.grid_points(n)
    ud = o.direct(gx, gy, q, gx[idx], gy[idx], o.self_log(n))
    err = np.linalg.norm(ug[idx] - ud) / np.linalg.norm(ud)
    say("  rel L2 err at 512 sampled nodes %.3e" % err)
    assert err <= 2e-6
