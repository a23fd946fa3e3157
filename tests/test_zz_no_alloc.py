"""The allocation-free bump-gradient entry point (fmm_bumps_grad_noalloc)
against fmm_bumps_grad, through the C ABI: two calls in a row on one device,
the second with a smaller input (smaller grid, fewer bumps), each equal to
the allocating entry point's result (the same kernels in the same order, so
bit for bit; the bar below is the oracle-parity bar of the bump gradients,
1e-12 relative).  Sizes beyond the static workspace are rejected."""
import sys

import numpy as np
import pytest

from paper_1308_3339_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _grads(fn, plan, K, seed):
    import torch
    cx, cy, w, a = (dev(v) for v in inputs.bump_params(K, seed=seed))
    g = dev(inputs.random_charges(plan.npts, seed=seed + 1))
    outs = [torch.full((K,), np.nan, dtype=torch.float64, device="cuda") for _ in range(4)]
    fn(plan, cx, cy, w, a, g, *outs)
    torch.cuda.synchronize()
    return np.stack([t.cpu().numpy() for t in outs])


def test_noalloc_matches_allocating_entry_point_twice():
    import paper_1308_3339_amd as fp
    cases = [(256, 200, 31), (64, 5, 32)]   # (n, K, seed): the second call is smaller
    for n, K, seed in cases:
        say("case bumps_grad_noalloc n=%d K=%d" % (n, K))
        with fp.fmm_setup(n=n, p=6, bem=0) as plan:
            got = _grads(fp.fmm_bumps_grad_noalloc, plan, K, seed)
            ref = _grads(fp.fmm_bumps_grad, plan, K, seed)
        assert np.all(np.isfinite(got))
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        say("  max rel diff vs fmm_bumps_grad %.3e, bitwise %s" % (err, np.array_equal(got, ref)))
        assert err <= 1e-12
        assert np.array_equal(got, ref)


def test_noalloc_rejects_more_bumps_than_the_workspace_holds():
    import torch

    import paper_1308_3339_amd as fp
    K = 257
    say("case bumps_grad_noalloc K=257 rejected")
    with fp.fmm_setup(n=64, p=6, bem=0) as plan:
        v = torch.ones(K, dtype=torch.float64, device="cuda")
        g = torch.zeros(plan.npts, dtype=torch.float64, device="cuda")
        with pytest.raises(fp.FmmError) as ei:
            fp.fmm_bumps_grad_noalloc(plan, v, v, v, v, g, v, v, v, v)
        assert ei.value.code == fp.FMM_ERR_ARG
        assert "256" in str(ei.value)
