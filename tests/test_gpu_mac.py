"""GPU parity of the MAC-theta path (Sec. 5.2 dual tree traversal on the
uniform tree) against the oracle's traversal, through the C ABI.

  * volume potential (fmm_apply, bem = 0) against the oracle's traversal FMM
    on the same seeded charges: max relative error <= 1e-12 (the tolerance
    of the list-rule path: FP64 end to end, different summation orders),
    over near radii K = 2, 3, 4, several p, grids of 1 to 32x32 leaves;
  * preconditioner stages (ring potential, boundary density, z) against the
    oracle's preconditioner with the same theta: 1e-12 / 1e-11 / 1e-11;
  * theta > 1/sqrt(2) reproduces the list rule bitwise (same tables, same
    kernels);
  * accuracy against the exact sum (about six digits at p = 6, theta = 0.4)
    and a solve against the oracle's (solution within 1e-6, true residual
    <= 1e-8 recomputed on the CPU, iterations within one);
  * point clouds with a MAC theta against the oracle's traversal FMM (1e-12),
    and more accurate than the list rule at the same p;
  * full size (2048^2, p = 6, theta = 0.4, the configuration bench.py times):
    charges in one leaf give the exact lattice sum at every node of the near
    disk around it; 512 sampled nodes against the direct sum within the
    truncation error; the solve reaches 1e-8.
"""
import math
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


@pytest.mark.parametrize("n,p,theta", [(8, 6, 0.4), (16, 6, 0.4), (32, 6, 0.4), (64, 6, 0.4),
                                       (64, 8, 0.3), (128, 6, 0.4), (128, 10, 0.3),
                                       (128, 12, 0.45), (256, 6, 0.4), (256, 9, 0.6),
                                       (64, 2, 0.5)])
def test_fmm_apply_theta_matches_oracle(n, p, theta):
    import paper_1308_3339_amd as fp
    say("case theta fmm_apply n=%d p=%d theta=%g" % (n, p, theta))
    q = inputs.random_charges(n * n, seed=500 + n + p)
    with fp.fmm_setup(n=n, p=p, bem=0, theta=theta) as plan:
        u = empty(n * n)
        plan.apply(dev(q), u)
        ug = host(u)
    uo = o.grid_fmm(n, p, q, theta=theta)
    err = relmax(ug, uo)
    say("  max rel err vs oracle traversal FMM %.3e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("n,p,theta", [(16, 6, 0.4), (32, 6, 0.4), (64, 6, 0.4), (128, 8, 0.3),
                                       (128, 6, 0.6), (256, 6, 0.4), (512, 6, 0.4)])
def test_precond_stages_theta_match_oracle(n, p, theta):
    import paper_1308_3339_amd as fp
    say("case theta precond stages n=%d p=%d theta=%g" % (n, p, theta))
    r = inputs.random_charges(n * n, seed=600 + n)
    with fp.fmm_setup(n=n, p=p, bem=1, theta=theta) as plan:
        z, phi, sig = empty(n * n), empty(4 * n), empty(4 * n)
        plan.precond_stages(dev(r), z, phi, sig)
        zg, phig, sigg = host(z), host(phi), host(sig)
        z2 = empty(n * n)
        plan.precond_apply(dev(r), z2)
        assert np.array_equal(host(z2), zg)
    zo, phio, sigo = o.Preconditioner(n, p=p, theta=theta).apply(r, stages=True)
    e_phi, e_sig, e_z = relmax(phig, phio), relmax(sigg, sigo), relmax(zg, zo)
    say("  phi_ring %.2e sigma %.2e z %.2e" % (e_phi, e_sig, e_z))
    assert e_phi <= 1e-12
    assert e_sig <= 1e-11
    assert e_z <= 1e-11


def test_large_theta_is_the_list_rule_bitwise():
    import paper_1308_3339_amd as fp
    n, p = 128, 8
    say("case theta 0.8 vs list rule")
    r = inputs.random_charges(n * n, seed=9)
    out = []
    for theta in (0.0, 0.8):
        with fp.fmm_setup(n=n, p=p, bem=1, theta=theta) as plan:
            z = empty(n * n)
            plan.precond_apply(dev(r), z)
            out.append(host(z))
    assert np.array_equal(out[0], out[1])


def test_theta_accuracy_against_exact_sum():
    import paper_1308_3339_amd as fp
    n = 256
    say("case theta accuracy n=256")
    q = inputs.random_charges(n * n, seed=7)
    ue = o.grid_direct_fft(n, q)
    errs = {}
    for p, theta in ((6, 0.0), (6, 0.4), (4, 0.4), (8, 0.3)):
        with fp.fmm_setup(n=n, p=p, bem=0, theta=theta) as plan:
            u = empty(n * n)
            plan.apply(dev(q), u)
            errs[(p, theta)] = np.linalg.norm(host(u) - ue) / np.linalg.norm(ue)
    say("  rel L2 errors", {k: "%.2e" % v for k, v in errs.items()})
    assert errs[(6, 0.4)] <= 1e-6
    assert errs[(6, 0.4)] < errs[(6, 0.0)] / 10
    assert errs[(8, 0.3)] < errs[(6, 0.4)]


@pytest.mark.parametrize("n", [64, 256])
def test_theta_solve_matches_oracle(n):
    import torch

    import paper_1308_3339_amd as fp
    say("case theta solve n=%d" % n)
    f = inputs.gaussian_bumps(n, 16, seed=700 + n)
    with fp.fmm_setup(n=n, p=6, theta=0.4) as plan:
        u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
        info = plan.solve(dev(f), u)
        ug = host(u)
    say("  info", info)
    assert info["converged"]
    res = np.linalg.norm(f - o.stencil(n, ug)) / np.linalg.norm(f)
    assert res <= 1e-8
    xo, io = o.fgmres(n, f, o.Preconditioner(n, p=6, theta=0.4))
    say("  iterations gpu %d oracle %d" % (info["iters"], io["iters"]))
    assert abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(ug - xo) <= 1e-6 * np.linalg.norm(xo)


def _levels(N):
    L = 0
    while (64 << (2 * L)) < N:
        L += 1
    return L


@pytest.mark.parametrize("N,p,theta", [(300, 8, 0.4), (5000, 10, 0.55), (8192, 6, 0.4),
                                       (20000, 8, 0.3)])
def test_points_theta_match_oracle(N, p, theta):
    """Point clouds (u_i = sum_{j != i} q_j G) with the traversal's near disk
    and lists: against the oracle's traversal FMM (1e-12) and, more accurate
    than the list rule at the same p, against the direct sum."""
    import torch

    import paper_1308_3339_amd as fp
    say("case theta points N=%d p=%d theta=%g" % (N, p, theta))
    x, y, q = inputs.random_points(N, seed_xy=800 + N, seed_q=900 + N)
    out = {}
    for th in (theta, 0.0):
        with fp.fmm_setup(kind=fp.FMM_POINTS, n=N, p=p, x=dev(x), y=dev(y), theta=th) as plan:
            u = torch.empty(N, dtype=torch.float64, device="cuda")
            plan.apply(dev(q), u)
            out[th] = host(u)
    uo = o.fmm(_levels(N), 0.0, 0.0, 1.0, p, x, y, q, x, y, 0.0, theta=theta)
    err = relmax(out[theta], uo)
    say("  max rel err vs oracle traversal FMM %.3e" % err)
    assert err <= 1e-12
    if _levels(N) >= 2:
        ud = o.direct(x, y, q, x, y, 0.0)
        e_t = np.linalg.norm(out[theta] - ud) / np.linalg.norm(ud)
        e_l = np.linalg.norm(out[0.0] - ud) / np.linalg.norm(ud)
        say("  rel L2 vs direct: theta %.2e, list rule %.2e" % (e_t, e_l))
        assert e_t < e_l


@pytest.fixture(scope="module")
def big_plan():
    import paper_1308_3339_amd as fp
    say("setup n=2048 p=6 theta=0.4")
    pl = fp.fmm_setup(n=2048, p=6, bem=0, theta=0.4)
    yield pl
    pl.close()


def test_fullsize_near_disk_is_exact(big_plan):
    n, K = 2048, 3
    say("case theta fullsize near disk")
    rng = np.random.default_rng(31)
    Lx, Ly = 97, 141     # source leaf
    q = np.zeros((n, n))
    q[8 * Ly:8 * Ly + 8, 8 * Lx:8 * Lx + 8] = rng.standard_normal((8, 8))
    q = q.reshape(-1)
    u = empty(n * n)
    big_plan.apply(dev(q), u)
    ug = host(u).reshape(n, n)
    src = np.flatnonzero(q)
    gx, gy = o.grid_points(n)
    lim = 2.0 / 0.4 ** 2
    near_t = []
    for b in range(-K, K + 1):
        for a in range(-K, K + 1):
            if a * a + b * b <= lim:
                tl = (Ly + b) * 8 * n + (Lx + a) * 8
                near_t.extend(tl + j * n + i for j in range(8) for i in range(8))
    near_t = np.array(near_t)
    ud = o.direct(gx[src], gy[src], q[src], gx[near_t], gy[near_t], o.self_log(n))
    e = np.abs(ug.reshape(-1)[near_t] - ud).max() / np.abs(ud).max()
    say("  near disk (%d nodes) max rel err %.2e" % (len(near_t), e))
    assert e <= 1e-13


def test_fullsize_sampled_against_direct(big_plan):
    n = 2048
    say("case theta fullsize sampled")
    q = inputs.random_charges(n * n, seed=77)
    u = empty(n * n)
    big_plan.apply(dev(q), u)
    ug = host(u)
    idx = inputs.target_subset(n * n, 512, seed=78)
    gx, gy = o.grid_points(n)
    ud = o.direct(gx, gy, q, gx[idx], gy[idx], o.self_log(n))
    err = np.linalg.norm(ug[idx] - ud) / np.linalg.norm(ud)
    say("  rel L2 err at 512 sampled nodes %.3e" % err)
    assert err <= 2e-6


def test_fullsize_theta_solve():
    import torch

    import paper_1308_3339_amd as fp
    n = 2048
    say("case theta fullsize solve")
    f = inputs.gaussian_bumps(n, 16, seed=inputs.SEED_BUMPS_2048)
    with fp.fmm_setup(n=n, p=6, theta=0.4) as plan:
        u = torch.zeros(n * n, dtype=torch.float64, device="cuda")
        info = plan.solve(dev(f), u)
        ug = host(u)
    say("  info", info)
    assert info["converged"] and info["iters"] <= 15
    res = np.linalg.norm(f - o.stencil(n, ug)) / np.linalg.norm(f)
    say("  CPU-recomputed true rel res %.3e" % res)
    assert res <= 1e-8
