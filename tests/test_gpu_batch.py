"""Batched uneven solves (precond_gmres_solve_batch) and the autotuner.

  * a mixed-size batch gives, per instance, bitwise the solution of the
    same plan's single solve (same kernels, fixed-order reductions), with
    and without HIP-graph replay of the Arnoldi steps, and again on a
    second and third batch (graphs replayed, eager work in between);
  * one instance against the oracle's solve;
  * the tuned vector-kernel block count is one of the candidates and keeps
    solutions within rounding of the untuned ones;
  * the 64-instance workload (16 each of 128^2, 256^2, 512^2, 1024^2,
    bumps seeded 1000 + k) converges to a true residual <= 1e-8 everywhere;
  * FP64, FP32 and split-FP16 plans of the 2048^2 workload in one batch all
    reach the FP64 true residual and agree with the FP64 solution.
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


SIZES = (64, 128, 32, 256, 64, 128)


def _setup(sizes, p=10):
    import paper_1308_3339_amd as fp
    plans = [fp.fmm_setup(n=n, p=p) for n in sizes]
    fs = [dev(inputs.gaussian_bumps(n, 16, seed=900 + i)) for i, n in enumerate(sizes)]
    return plans, fs


def test_batch_equals_single_solves_and_replays():
    import torch

    import paper_1308_3339_amd as fp
    say("case batch vs single, sizes", SIZES)
    plans, fs = _setup(SIZES)
    try:
        single = []
        for pl, f in zip(plans, fs):
            u = torch.zeros_like(f)
            info = pl.solve(f, u)
            assert info["converged"]
            single.append((host(u), info["iters"]))
        for graphs in (False, True, True, True):
            us = [torch.zeros_like(f) for f in fs]
            out = fp.precond_gmres_solve_batch(plans, fs, us, graphs=graphs)
            assert out["status"] == fp.FMM_OK
            for i, (u, r) in enumerate(zip(us, out["results"])):
                assert r["iters"] == single[i][1]
                assert np.array_equal(host(u), single[i][0]), (graphs, i)
            say("  graphs=%s iters" % graphs, [r["iters"] for r in out["results"]],
                "elapsed ms", [round(e, 2) for e in out["elapsed_ms"]])
            # eager work on the same plans between replays
            w = torch.empty_like(fs[0])
            plans[0].precond_apply(fs[0], w)
    finally:
        for pl in plans:
            pl.close()


def test_batch_instance_matches_oracle():
    import torch

    import paper_1308_3339_amd as fp
    say("case batch vs oracle")
    plans, fs = _setup((32, 64))
    try:
        us = [torch.zeros_like(f) for f in fs]
        fp.precond_gmres_solve_batch(plans, fs, us)
        n = 64
        xo, _ = o.fgmres(n, host(fs[1]), o.Preconditioner(n, p=10))
        ug = host(us[1])
        assert np.linalg.norm(ug - xo) <= 1e-6 * np.linalg.norm(xo)
        res = np.linalg.norm(host(fs[1]) - o.stencil(n, ug)) / np.linalg.norm(host(fs[1]))
        assert res <= 1e-8
    finally:
        for pl in plans:
            pl.close()


def test_tuner_choice_and_solutions():
    import torch

    import paper_1308_3339_amd as fp
    say("case tuner")
    for n in (128, 1024):
        with fp.fmm_setup(n=n, p=10) as pl:
            f = dev(inputs.gaussian_bumps(n, 16, seed=910 + n))
            u0 = torch.zeros_like(f)
            pl.solve(f, u0)
            nb = pl.tune()
            say("  n=%d tuned vector blocks %d" % (n, nb))
            assert nb in (64, 128, 256, 512, 1024, 2048, 4096)
            u1 = torch.zeros_like(f)
            info = pl.solve(f, u1)
            assert info["converged"]
            a, b = host(u0), host(u1)
            assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()


def test_batch_rejects_bad_arguments():
    import torch

    import paper_1308_3339_amd as fp
    plans, fs = _setup((32,))
    try:
        u = torch.zeros_like(fs[0])
        with pytest.raises(fp.FmmError):
            fp.precond_gmres_solve_batch([plans[0], plans[0]], [fs[0], fs[0]], [u, torch.zeros_like(u)])
        with pytest.raises(fp.FmmError):
            fp.precond_gmres_solve_batch(plans, fs, [fs[0]])
        with pytest.raises(ValueError):
            fp.precond_gmres_solve_batch(plans, fs, [])
    finally:
        for pl in plans:
            pl.close()


def test_batch_64_uneven_instances():
    import torch

    import paper_1308_3339_amd as fp
    sizes = [s for s in (128, 256, 512, 1024) for _ in range(16)]
    say("case batch 64 instances")
    plans = [fp.fmm_setup(n=n, p=10) for n in sizes]
    try:
        fs = [dev(inputs.gaussian_bumps(n, 16, seed=1000 + k)) for k, n in enumerate(sizes)]
        us = [torch.zeros_like(f) for f in fs]
        out = fp.precond_gmres_solve_batch(plans, fs, us)
        assert out["status"] == fp.FMM_OK
        worst = 0.0
        for pl, f, u in zip(plans, fs, us):
            w = torch.empty_like(u)
            pl.stencil_apply(u, w)
            worst = max(worst, float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f)))
        el = np.array(out["elapsed_ms"])
        say("  worst true rel res %.2e; iters %s; p50 %.2f ms p99 %.2f ms" %
            (worst, sorted(set(r["iters"] for r in out["results"])), np.percentile(el, 50),
             np.percentile(el, 99)))
        assert worst <= 1e-8
    finally:
        for pl in plans:
            pl.close()


def test_reduced_precision_batch_at_2048_reaches_fp64_residual():
    """The split-FP16 and FP32 plans in one batch with an FP64 plan on 2048^2
    grids: every instance reaches the FP64 true residual 1e-8 and the reduced
    solutions agree with the FP64 one within the 1e-6 solution bar."""
    import torch

    import paper_1308_3339_amd as fp
    n = 2048
    say("case batch 2048 fp64 + fp32 + split-fp16")
    precs = (fp.FMM_FP64, fp.FMM_FP32, fp.FMM_SPLIT_FP16)
    plans = [fp.fmm_setup(n=n, p=10, prec=pr) for pr in precs]
    try:
        f = dev(inputs.gaussian_bumps(n, 16, seed=inputs.SEED_BUMPS_2048))
        fs = [f, f.clone(), f.clone()]
        us = [torch.zeros_like(f) for _ in precs]
        out = fp.precond_gmres_solve_batch(plans, fs, us)
        assert out["status"] == fp.FMM_OK
        ref = us[0]
        for pl, u, r in zip(plans, us, out["results"]):
            w = torch.empty_like(u)
            pl.stencil_apply(u, w)
            res = float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f))
            diff = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(ref))
            say("  iters %d true rel res %.2e  rel diff vs fp64 %.2e" % (r["iters"], res, diff))
            assert res <= 1e-8 and diff <= 1e-6
    finally:
        for pl in plans:
            pl.close()
