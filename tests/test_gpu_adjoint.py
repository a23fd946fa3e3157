"""Differentiation through the FMM-preconditioned solve, through the C ABI.

  * bump source and its parameter gradients against the oracle (1e-12);
  * the adjoint solve against the exact discrete solve (sine transform);
  * the 1024^2 workload: L = 0.5 |u - u_t|^2, u the solve for a 16-bump
    source (seed 7), u_t the solve for an 8-bump source (seed 6); gradients
    with respect to f at 32 seeded nodes (seed 8) and with respect to the 16
    bump centres, from torch.autograd over the library's adjoint, against
    the oracle's exact gradients and against central differences (h = 1e-6,
    FP64) of the oracle's exact loss, relative error <= 1e-5.
"""
import sys

import numpy as np
import pytest

from oracle import adjoint as adj
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
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,K", [(64, 16), (1024, 16), (128, 1)])
def test_bumps_eval_and_grad_match_oracle(n, K):
    import torch

    import paper_1308_3339_amd as fp
    say("case bumps n=%d K=%d" % (n, K))
    cx, cy, w, a = inputs.bump_params(K, seed=40 + n)
    g = np.random.default_rng(41).standard_normal(n * n)
    with fp.fmm_setup(n=n, p=8, bem=0) as plan:
        f = torch.empty(n * n, dtype=torch.float64, device="cuda")
        plan.bumps_eval(dev(cx), dev(cy), dev(w), dev(a), f)
        outs = [torch.empty(K, dtype=torch.float64, device="cuda") for _ in range(4)]
        plan.bumps_grad(dev(cx), dev(cy), dev(w), dev(a), dev(g), *outs)
        fg = host(f)
        grads = [host(t) for t in outs]
    fo = adj.bumps_eval(n, cx, cy, w, a)
    go = adj.bumps_grad(n, cx, cy, w, a, g)
    e = relmax(fg, fo)
    eg = max(relmax(x, y) for x, y in zip(grads, go))
    say("  f rel err %.2e, grad rel err %.2e" % (e, eg))
    assert e <= 1e-13
    assert eg <= 1e-12


def test_bumps_reject_bad_counts():
    import torch

    import paper_1308_3339_amd as fp
    with fp.fmm_setup(n=32, p=6, bem=0) as plan:
        f = torch.empty(32 * 32, dtype=torch.float64, device="cuda")
        z = torch.zeros(0, dtype=torch.float64, device="cuda")
        with pytest.raises(fp.FmmError):
            plan.bumps_eval(z, z, z, z, f)
        big = torch.ones(257, dtype=torch.float64, device="cuda")
        with pytest.raises(fp.FmmError):
            plan.bumps_eval(big, big, big, big, f)


@pytest.mark.parametrize("n", [128, 512])
def test_adjoint_solve_matches_exact_solve(n):
    import torch

    import paper_1308_3339_amd as fp
    say("case adjoint solve n=%d" % n)
    g = inputs.gaussian_bumps(n, 16, seed=50 + n)
    with fp.fmm_setup(n=n, p=10) as plan:
        lam = torch.zeros(n * n, dtype=torch.float64, device="cuda")
        info = plan.solve_adjoint(dev(g), lam, tol=1e-10)
        lg = host(lam)
    say("  info", info)
    assert info["converged"]
    e = relmax(lg, adj.fd_solve_exact(n, g))
    say("  rel err vs exact solve %.2e" % e)
    assert e <= 1e-8


def test_config5_gradients_against_oracle_and_central_differences():
    import torch

    import paper_1308_3339_amd as fp
    from paper_1308_3339_amd.autograd import gaussian_bumps, poisson_solve
    n = 1024
    tol = 1e-10
    say("case config5 n=1024")
    tcx, tcy, tw, ta = inputs.bump_params(8, seed=inputs.SEED_ADJ_TARGET)
    cx, cy, w, a = inputs.bump_params(16, seed=inputs.SEED_ADJ_SOURCE)
    idx = inputs.target_subset(n * n, 32, seed=inputs.SEED_ADJ_COORDS)
    with fp.fmm_setup(n=n, p=10) as plan:
        with torch.no_grad():
            ft = gaussian_bumps(plan, dev(tcx), dev(tcy), dev(tw), dev(ta))
            u_t = poisson_solve(plan, ft, tol=tol)
        pcx, pcy = dev(cx).requires_grad_(True), dev(cy).requires_grad_(True)
        f = gaussian_bumps(plan, pcx, pcy, dev(w), dev(a))
        f.retain_grad()
        u = poisson_solve(plan, f, tol=tol)
        loss = 0.5 * ((u - u_t) ** 2).sum()
        loss.backward()
        gf, gcx, gcy = host(f.grad), host(pcx.grad), host(pcy.grad)
        Lg = float(loss.detach().cpu())
    # oracle: exact solves, its own u_t
    fo = adj.bumps_eval(n, cx, cy, w, a)
    uto = adj.fd_solve_exact(n, adj.bumps_eval(n, tcx, tcy, tw, ta))
    Lo = adj.loss(n, fo, uto)
    lam = adj.loss_grad_f(n, fo, uto)
    ocx, ocy, _, _ = adj.bumps_grad(n, cx, cy, w, a, lam)
    say("  loss gpu %.12e oracle %.12e" % (Lg, Lo))
    assert abs(Lg - Lo) <= 1e-8 * Lo
    e_f = relmax(gf[idx], lam[idx])
    e_c = max(relmax(gcx, ocx), relmax(gcy, ocy))
    say("  grad f (32 nodes) rel err vs oracle %.2e; grad centres %.2e" % (e_f, e_c))
    assert e_f <= 1e-5 and e_c <= 1e-5
    # central differences (h = 1e-6) of the oracle's exact loss
    fd_f = adj.central_fd_f(n, fo, uto, idx, h=1e-6)
    fd_cx, fd_cy = adj.central_fd_centres(n, cx, cy, w, a, uto, h=1e-6)
    e_fdf = relmax(gf[idx], fd_f)
    e_fdc = max(relmax(gcx, fd_cx), relmax(gcy, fd_cy))
    say("  vs central differences: grad f %.2e, grad centres %.2e" % (e_fdf, e_fdc))
    assert e_fdf <= 1e-5 and e_fdc <= 1e-5
