#!/usr/bin/env python3
"""Benchmark of the FMM-preconditioned Krylov solve on one MI355X.

Workload (one "step"): precond_gmres_solve of the 5-point FD Poisson matrix
on a 2048 x 2048 interior grid of the unit square, zero Dirichlet data,
f = 16 seeded Gaussian bumps, FMM-BEM preconditioner with p = 10 and 8x8
leaves, FGMRES(30) to a 1e-8 true relative residual, all in FP64.  Setup
(tree tables, boundary inverse) is done once before the warmup and reported
separately.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Also reports the bare FMM throughput (Mpoints/s),
a per-stage breakdown with each stage against its own bound, the roofline of
the dominant kernel (the leaf kernel: near field and P2M, timed with HIP
events on the library's stream over the timed region) and the CPU oracle on
a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_leaf_grid_2048_p10_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def leaf_kernel_flops(n, p):
    """Algorithmic flops of one k_leaf_grid launch on an n x n grid: every
    near-field pair (target, source in the 3x3 leaves) is one multiply-add
    (2 flops); every source point adds to the p complex coefficients of its
    leaf's multipole expansion (2 multiply-adds per coefficient, 4p flops)."""
    nl = n // 8
    pairs = 4096 * (3 * nl - 2) ** 2
    return 2.0 * pairs + 4.0 * p * n * n


PEAK_HBM_TBS = 8.0             # MI355X HBM3E
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector (packed FP32 issue)


def m2l_translations(L):
    """M2L translations of one application on the uniform tree with the list rule
    (children of the parent's 3x3 neighbourhood minus the own 3x3 block, cut at
    the domain edge), levels 2..L."""
    return sum(16 * (3 * 2 ** (l - 1) - 2) ** 2 - (3 * 2 ** l - 2) ** 2 for l in range(2, L + 1))


def stage_rooflines(n, p, prof):
    """Each timed stage of one solve against its own bound.  prof maps a stage to
    (ms per solve, timed calls per solve: one per application or Arnoldi step).  Algorithmic work per launch:
      LEAF    leaf_kernel_flops (near-field pairs + P2M), FP64 VALU;
      M2L     8 p^2 flops per translation (p^2 complex multiply-adds), FP64 VALU;
      BEM     the eight folded (n/2)^2 FP64 halves of the boundary inverse, HBM;
      ARNOLDI step j reads z, v_0..v_j twice and writes two vectors: (2j+6) 8N bytes, HBM;
      PASS2   the final sweep over the grid: z read and written (16 N bytes) and the
              leaf-level local expansions of both passes read (2 x 16 p bytes per
              leaf); the ring-source kernels before it touch only the boundary band, HBM;
      STENCIL a residual r = b - A x reads b and x and writes r: 24 N bytes, HBM.
    The tree passes (M2M, L2L, RING) are bound by the latency of their dependent
    steps; only their time is given."""
    L = (n // 8).bit_length() - 1
    N = n * n
    out = {}
    for name, (ms, cnt) in prof.items():
        if not cnt or ms <= 0:
            continue
        sec = ms * 1e-3
        if name == "LEAF":
            work, unit, peak, bound = leaf_kernel_flops(n, p) * cnt / 1e12, "TFLOP/s", PEAK_FP64_VALU_TFLOPS, "alu"
        elif name == "M2L":
            work, unit, peak, bound = 8.0 * p * p * m2l_translations(L) * cnt / 1e12, "TFLOP/s", PEAK_FP64_VALU_TFLOPS, "alu"
        elif name == "BEM":
            work, unit, peak, bound = 8.0 * (n // 2) ** 2 * 8 * cnt / 1e12, "TB/s", PEAK_HBM_TBS, "hbm"
        elif name == "ARNOLDI":
            work, unit, peak, bound = sum((2 * j + 6) * 8.0 * N for j in range(cnt)) / 1e12, "TB/s", PEAK_HBM_TBS, "hbm"
        elif name == "PASS2":
            nleaf = (n // 8) ** 2
            work, unit, peak, bound = (16.0 * N + 2 * 16.0 * p * nleaf) * cnt / 1e12, "TB/s", PEAK_HBM_TBS, "hbm"
        elif name == "STENCIL":
            work, unit, peak, bound = 24.0 * N * cnt / 1e12, "TB/s", PEAK_HBM_TBS, "hbm"
        else:
            out[name] = {"ms_per_solve": round(ms, 4), "calls": cnt, "bound": "latency"}
            continue
        ach = work / sec
        out[name] = {"ms_per_solve": round(ms, 4), "calls": cnt, "bound": bound, "achieved": round(ach, 3),
                     "unit": unit, "peak": peak, "frac": round(ach / peak, 4)}
    return out


def leaf_kernel_hash():
    """sha256 of the source text of k_leaf_grid (from its template line to the
    closing brace), so that only a change of that kernel invalidates the
    committed counter summary."""
    src = open(os.path.join(ROOT, "paper_1308_3339_amd", "csrc", "fmm_grid.hip")).read()
    i = src.rindex("\n", 0, src.index(" void k_leaf_grid(LeafArgs a)")) + 1
    j = src.index("\n}\n", i)
    return hashlib.sha256(src[i:j].encode()).hexdigest()


def kernel_source_hash(fname, head):
    """sha256 of a kernel's source text, from the line that declares it to the
    closing brace of its body."""
    src = open(os.path.join(ROOT, "paper_1308_3339_amd", "csrc", fname)).read()
    i = src.index(head)
    j = src.index("\n}\n", i)
    return hashlib.sha256(src[i:j].encode()).hexdigest()


POINTS_ISA_FILE = os.path.join(ROOT, "profiles", "k_leaf_points_isa.md")
POINTS_HEADS = {"fp64": ("points.hip", "__global__ __launch_bounds__(256) void k_leaf_points("),
                "fp32": ("points.hip", "__global__ __launch_bounds__(256) void k_leaf_points_f32(")}


def points_isa_counts():
    """VALU instructions per near-field pair of the point leaf kernels, from the
    committed count of their inner loops in the AMD assembly, when it was taken
    on the current kernel sources ({kind: (valu, flops)} or {})."""
    if not os.path.exists(POINTS_ISA_FILE):
        return {}
    txt = open(POINTS_ISA_FILE).read()
    out = {}
    for kind, (fname, head) in POINTS_HEADS.items():
        m = re.search(r"%s_sha256:\s*([0-9a-f]{64})\s+%s_valu_per_pair:\s*(\d+)\s+%s_flops_per_pair:\s*(\d+)"
                      % (kind, kind, kind), txt)
        if m and m.group(1) == kernel_source_hash(fname, head):
            out[kind] = (int(m.group(2)), int(m.group(3)))
    return out


# VALU issue: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz lane-instructions per second
PEAK_VALU_TINSTR = 39.32


def traffic_from_profile(src_hash):
    """HBM bytes per leaf-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    m_f = re.search(r"fetch_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_w = re.search(r"write_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m_hash and m_f and m_w) or m_hash.group(1) != src_hash:
        return None
    return float(m_f.group(1)) + float(m_w.group(1))


def cpu_baseline(n, p, f):
    """The oracle (plain C, FP64, OpenMP over independent targets) on the same
    workload: its preconditioner setup (the LU factors of the 4n x 4n boundary
    matrix) timed on its own, one preconditioner application on the right-hand
    side (both FMM passes and the LU solve; its ring potential, boundary
    density and output are kept to measure the GPU plans against), and one
    whole right-preconditioned FGMRES(30) solve to 1e-8 (modified Gram-Schmidt
    Arnoldi, one preconditioner application per iteration), setup excluded.
    value = 1 / solve time."""
    import oracle as o
    t0 = time.perf_counter()
    pc = o.Preconditioner(n, p=p)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    zo, phio, sigo = pc.apply(f, stages=True)
    t_apply = time.perf_counter() - t0
    t0 = time.perf_counter()
    xo, info = o.fgmres(n, f, pc)
    t_solve = time.perf_counter() - t0
    pc.close()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"value": 1.0 / t_solve, "unit": "solves/s", "cores": o.max_threads(), "kind": "oracle",
           "cpu": model, "nproc": os.cpu_count(),
           "sample": "one whole oracle solve of the benchmark problem (%dx%d, p=%d, same f, "
                     "FGMRES(30) to 1e-8: %d iterations, %.2f s wall), its setup (boundary LU, "
                     "%.2f s) excluded; one oracle preconditioner application takes %.2f s"
                     % (n, n, p, info["iters"], t_solve, t_setup, t_apply),
           "setup_s": round(t_setup, 3), "precond_apply_s": round(t_apply, 3),
           "solve_s": round(t_solve, 3), "iters": info["iters"],
           "true_rel_res": info["true_rel_res"]}
    return out, {"z": zo, "phi": phio, "sigma": sigo, "x": xo}


def adjoint_block(fp, inputs, torch, steps, warmup):
    """Differentiation workload on a 1024 x 1024 grid: L = 0.5 |u - u_t|^2 with
    u the solve for a 16-bump source (seed 7) and u_t for an 8-bump source
    (seed 6).  Times one gradient (bump source, forward solve, loss, adjoint
    solve, bump-parameter gradients) and checks the centre gradients against
    central differences (h = 1e-6) of the same GPU loss, each difference
    evaluated as (u+ - u-) . ((u+ + u-)/2 - u_t)."""
    from paper_1308_3339_amd.autograd import gaussian_bumps, poisson_solve
    n, tol, h = 1024, 1e-10, 1e-6
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(a).to(dev)
    tcx, tcy, tw, ta = (T(v) for v in inputs.bump_params(8, seed=inputs.SEED_ADJ_TARGET))
    cx, cy, w, a = (T(v) for v in inputs.bump_params(16, seed=inputs.SEED_ADJ_SOURCE))
    plan = fp.fmm_setup(n=n, p=10, bem=1)
    with torch.no_grad():
        u_t = poisson_solve(plan, gaussian_bumps(plan, tcx, tcy, tw, ta), tol=tol)

    def gradient():
        pcx, pcy = cx.clone().requires_grad_(True), cy.clone().requires_grad_(True)
        u = poisson_solve(plan, gaussian_bumps(plan, pcx, pcy, w, a), tol=tol)
        (0.5 * ((u - u_t) ** 2).sum()).backward()
        return pcx.grad, pcy.grad

    for _ in range(warmup):
        gradient()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gx, gy = gradient()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps

    def u_of(cxv, cyv):
        with torch.no_grad():
            return poisson_solve(plan, gaussian_bumps(plan, cxv, cyv, w, a), tol=tol)

    fd = torch.zeros(2, 16, dtype=torch.float64, device=dev)
    for k in range(16):
        for c, (base, other) in enumerate(((cx, cy), (cy, cx))):
            bp, bm = base.clone(), base.clone()
            bp[k] += h
            bm[k] -= h
            up, um = (u_of(bp, other), u_of(bm, other)) if c == 0 else (u_of(other, bp), u_of(other, bm))
            fd[c, k] = torch.dot(up - um, 0.5 * (up + um) - u_t) / (2 * h)
    g = torch.stack([gx, gy])
    err = float((g - fd).abs().max() / g.abs().max())
    plan.close()
    return {"workload": "1024x1024 grid, L = 0.5|u - u_t|^2, u: 16-bump source (seed %d), "
                        "u_t: 8-bump source (seed %d), solves to %.0e, p=10"
                        % (inputs.SEED_ADJ_SOURCE, inputs.SEED_ADJ_TARGET, tol),
            "gradients_per_s": round(1.0 / dt, 3), "ms_per_gradient": round(1000.0 * dt, 3),
            "centre_grad_rel_err_vs_central_fd": err,
            "fd": "central differences h=1e-6 of the GPU loss over the 32 centre coordinates"}


def varcoef_block(fp, inputs, torch, plan, f, steps, warmup):
    """Variable-coefficient problem of Sec. 6.4 on the same grid and source:
    -div(a grad u) = f, a = 1 + 2^-4 sin(4 pi X) sin(4 pi Y), preconditioned by
    the plan's constant-coefficient FMM-BEM operator."""
    n = plan.n
    mu, m = 2.0 ** -4, 4
    ax, ay = (torch.from_numpy(v).to(f.device) for v in inputs.var_faces(n, mu, m, m))
    u = torch.zeros_like(f)
    for _ in range(warmup):
        u.zero_()
        plan.solve_var(ax, ay, f, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        info = plan.solve_var(ax, ay, f, u)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    w = torch.empty_like(u)
    plan.stencil_var_apply(ax, ay, u, w)
    rel = float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f))
    return {"workload": "%dx%d grid, -div(a grad u) = f, a = 1 + mu sin(m pi X) sin(m pi Y), "
                        "mu = 2^-4, m = %d, same f, constant-coefficient FMM-BEM preconditioner"
                        % (n, n, m),
            "solves_per_s": round(1.0 / dt, 4), "ms_per_solve": round(1000.0 * dt, 4),
            "iters": info["iters"], "true_rel_res": rel}


def points_block(fp, inputs, torch, steps, warmup):
    """Point-cloud FMM (Sec. 5 on a uniform tree, list rule): 1,048,576 uniform
    random points in the unit square, charges U(-1, 1), p = 10, FP64 next to
    FMM_FP32 (near field pairwise in FP32 with the polynomial logarithm and
    Kahan sums, Secs. 5.3 and 7.1; far field FP64).  Near pairs counted from
    the leaf occupancy (every ordered pair of points in 3x3-adjacent leaves,
    self pairs excluded)."""
    import numpy as np
    N, p = 1 << 20, 10
    x, y, q = inputs.random_points(N)
    L = 0
    while (64 << (2 * L)) < N:
        L += 1
    nl = 1 << L
    ix = np.clip(np.floor(x * nl).astype(np.int64), 0, nl - 1)
    iy = np.clip(np.floor(y * nl).astype(np.int64), 0, nl - 1)
    cnt = np.bincount(iy * nl + ix, minlength=nl * nl).reshape(nl, nl).astype(np.float64)
    pad = np.pad(cnt, 1)
    near = sum(pad[1 + b:1 + b + nl, 1 + a:1 + a + nl] for b in (-1, 0, 1) for a in (-1, 0, 1))
    pairs = float((cnt * near).sum() - N)
    dev = torch.device("cuda:0")
    xd, yd, qd = (torch.from_numpy(v).to(dev) for v in (x, y, q))
    out = {}
    res = {}
    isa = points_isa_counts()
    for name, prec in (("fp64", fp.FMM_FP64), ("fp32", fp.FMM_FP32)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl = fp.fmm_setup(kind=fp.FMM_POINTS, n=N, p=p, x=xd, y=yd, prec=prec)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        with pl:
            u = torch.empty(N, dtype=torch.float64, device=dev)
            for _ in range(max(warmup, 1)):
                pl.apply(qd, u)
            pl.profile(("LEAF",))
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                pl.apply(qd, u)
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / steps
            lms, ln = pl.profile_read().get("LEAF", (0.0, 0))
            pl.profile(())
            leaf_ms = lms / max(ln, 1)
            res[name] = u.clone()
            gps = pairs / (leaf_ms * 1e-3)
            out[name] = {"apply_ms": round(ms, 4), "mpoints_per_s": round(N / (ms * 1e-3) / 1e6, 2),
                         "setup_s": round(setup_s, 4),
                         "leaf_ms": round(leaf_ms, 4),
                         "near_gpairs_per_s": round(gps / 1e9, 2)}
            if name in isa:
                valu, flops = isa[name]
                peak = PEAK_FP64_VALU_TFLOPS if name == "fp64" else PEAK_FP32_VALU_TFLOPS
                out[name]["leaf_roofline"] = {
                    "bound": "alu", "kernel": "k_leaf_points" + ("_f32" if name == "fp32" else ""),
                    "flops_per_pair": flops, "achieved": round(gps * flops / 1e12, 3),
                    "unit": "TFLOP/s", "peak": peak, "frac": round(gps * flops / 1e12 / peak, 4),
                    "valu_instr_per_pair": valu,
                    "valu_issue_frac": round(gps * valu / 1e12 / PEAK_VALU_TINSTR, 4)}
    diff = float((res["fp32"] - res["fp64"]).abs().max() / res["fp64"].abs().max())
    return {"workload": "%d uniform random points in the unit square (seeds %d, %d), q ~ U(-1,1), "
                        "p=%d, list rule, L=%d" % (N, inputs.SEED_POINTS_XY, inputs.SEED_POINTS_Q, p, L),
            "near_pairs": pairs, "fp64": out["fp64"], "fp32": out["fp32"],
            "fp32_max_rel_diff_vs_fp64": diff,
            "fp32_speedup": round(out["fp64"]["apply_ms"] / out["fp32"]["apply_ms"], 3)}


def direct_sum_sampled(torch, n, q, idx, dev):
    """Exact grid sum u_i = -(1/2pi) [sum_{j != i} q_j log(h |i - j|) + q_i log(eps_s h)]
    at the sampled nodes idx, in FP64 with plain torch operations (a reference
    for the measurement, not part of the measured path)."""
    h = 1.0 / (n + 1)
    eps_s = math.exp(-0.57721566490153286061) / (2.0 * math.sqrt(2.0))
    qd = torch.as_tensor(q, device=dev)
    jj = torch.arange(n * n, device=dev)
    gx = ((jj % n) + 1).to(torch.float64) * h
    gy = ((jj // n) + 1).to(torch.float64) * h
    out = []
    for i in idx:
        r2 = (gx - gx[i]) ** 2 + (gy - gy[i]) ** 2
        r2[i] = 1.0
        lg = 0.5 * torch.log(r2)
        lg[i] = math.log(eps_s * h)
        out.append(-(qd * lg).sum() / (2.0 * math.pi))
    return torch.stack(out).cpu().numpy()


def psweep_block(fp, inputs, torch, steps, warmup):
    """The plain FP64 method at 1024 x 1024 (16 bumps, seed 1) for p in
    {6, 8, 10, 12, 14}: solves/s to 1e-8, iterations, the bare FMM rate, and
    the FMM's error against the exact grid sum (relative L2 at 512 sampled
    nodes, random charges U(-1, 1), seed 77)."""
    import numpy as np
    n = 1024
    dev = torch.device("cuda:0")
    f = torch.from_numpy(inputs.gaussian_bumps(n, 16, seed=inputs.SEED_BUMPS_1024)).to(dev)
    qh = inputs.random_charges(n * n, seed=77)
    q = torch.from_numpy(qh).to(dev)
    idx = inputs.target_subset(n * n, 512, seed=78)
    ref = direct_sum_sampled(torch, n, qh, idx, dev)
    u = torch.zeros_like(f)
    w = torch.empty_like(f)
    rows = {}
    for p in (6, 8, 10, 12, 14):
        with fp.fmm_setup(n=n, p=p, bem=1) as pl:
            pl.tune()
            spl = pl.tune_m2l()
            for _ in range(max(warmup, 1)):
                u.zero_()
                pl.solve(f, u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                u.zero_()
                info = pl.solve(f, u)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            pl.stencil_apply(u, w)
            rel = float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f))
            uq = torch.empty_like(q)
            pl.apply(q, uq)
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(10):
                pl.apply(q, uq)
            e1.record(st)
            e1.synchronize()
            ams = e0.elapsed_time(e1) / 10
            ug = uq.cpu().numpy()[idx]
            err = float(np.linalg.norm(ug - ref) / np.linalg.norm(ref))
        rows[str(p)] = {"solves_per_s": round(1.0 / dt, 3), "ms_per_solve": round(1000 * dt, 4),
                        "iters": info["iters"], "true_rel_res": rel, "m2l_split": spl,
                        "fmm_apply_ms": round(ams, 4),
                        "fmm_mpoints_per_s": round(n * n / (ams * 1e-3) / 1e6, 1),
                        "fmm_rel_l2_err_vs_direct": err}
    return {"workload": "1024x1024 grid, f = 16 Gaussian bumps (seed %d), FMM-BEM preconditioner, "
                        "FGMRES(30) to 1e-8, FP64; FMM error on random charges (seed 77) at 512 "
                        "sampled nodes (seed 78) against the exact sum" % inputs.SEED_BUMPS_1024,
            "by_p": rows}


def batched_block(fp, inputs, torch, steps, warmup, prec=None):
    """64 independent solves of uneven sizes (16 each of 128^2, 256^2, 512^2,
    1024^2; instance k has 16 bumps seeded 1000 + k), p = 10, FGMRES(30) to
    1e-8.  Each plan's vector kernels are autotuned first.  The batch runs as
    four groups of 16 same-size instances (one launch per stage for a group,
    Givens rotations and convergence flags on the device), the steps and
    cycle ends replayed from HIP graphs captured in the warm-up.  Reports
    instances/s over the whole batch and the p50/p99 of the per-instance
    completion times, next to the batch without graphs, the separate layout
    (one solve per plan on its own stream, host Givens) and the same 64
    solves run one after another."""
    sizes = [s for s in (128, 256, 512, 1024) for _ in range(16)]
    dev = torch.device("cuda:0")
    plans = [fp.fmm_setup(n=n, p=10, bem=1, prec=fp.FMM_FP64 if prec is None else prec)
             for n in sizes]
    fs = [torch.from_numpy(inputs.gaussian_bumps(n, 16, seed=1000 + k)).to(dev)
          for k, n in enumerate(sizes)]
    us = [torch.zeros_like(f) for f in fs]
    tuned, splits = {}, {}
    for pl in plans:
        tuned[pl.n] = pl.tune()
        splits[pl.n] = pl.tune_m2l()

    def run(graphs, separate=False):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fp.precond_gmres_solve_batch(plans, fs, us, graphs=graphs, separate=separate)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    for _ in range(max(warmup, 1)):
        run(True)
    tg, el = [], []
    for _ in range(steps):
        t, out = run(True)
        tg.append(t)
        el.extend(out["elapsed_ms"])
    iters = [r["iters"] for r in out["results"]]
    ok = all(r["converged"] for r in out["results"])
    tn = min(run(False)[0] for _ in range(2))
    run(True, True)
    tsep = min(run(True, True)[0] for _ in range(2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, f, u in zip(plans, fs, us):
        u.zero_()
        pl.solve(f, u)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for pl in plans:
        pl.close()
    tbest = min(tg)
    el = sorted(el)
    pct = lambda q: el[min(len(el) - 1, int(round(q * (len(el) - 1))))]
    return {"workload": "64 instances: 16 each of 128^2, 256^2, 512^2, 1024^2, bumps seeded "
                        "1000+k, p=10, FGMRES(30) to 1e-8, FP64",
            "instances_per_s": round(64.0 / tbest, 2), "batch_ms": round(1000.0 * tbest, 3),
            "p50_ms": round(pct(0.5), 3), "p99_ms": round(pct(0.99), 3),
            "all_converged": ok, "iters_min_max": [min(iters), max(iters)],
            "no_graphs_instances_per_s": round(64.0 / tn, 2),
            "separate_plans_instances_per_s": round(64.0 / tsep, 2),
            "sequential_instances_per_s": round(64.0 / ts, 2),
            "tuned_vector_blocks": {str(k): v for k, v in sorted(tuned.items())},
            "tuned_m2l_split": {str(k): v for k, v in sorted(splits.items())}}


def trace_summary(path, top=40):
    """Markdown tables from a rocprofv3 kernel trace (csv): total, calls and
    average duration per kernel, then per kernel and launch shape (grid in
    threads) for the kernels of the FMM and Krylov stages."""
    import csv
    rows = list(csv.DictReader(open(path)))
    by_k, by_shape = {}, {}
    def short(name):
        # drop the argument list of a demangled kernel name
        depth, cut = 0, len(name)
        for i, ch in enumerate(name):
            if ch == "<":
                depth += 1
            elif ch == ">":
                depth -= 1
            elif ch == "(" and depth == 0:
                cut = i
                break
        return name[:cut]

    for r in rows:
        name = short(r["Kernel_Name"])
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
        shape = (int(r.get("Grid_Size_X", 0) or 0), int(r.get("Grid_Size_Y", 0) or 0))
        by_k.setdefault(name, []).append(dur)
        by_shape.setdefault((name, shape), []).append(dur)
    total = sum(sum(v) for v in by_k.values())
    out = ["| Kernel | Calls | Total us | Average us | % |", "|---|---:|---:|---:|---:|"]
    for name, v in sorted(by_k.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append("| `%s` | %d | %.1f | %.2f | %.2f |" % (name, len(v), sum(v), sum(v) / len(v),
                                                          100.0 * sum(v) / total))
    out += ["", "| Kernel | Grid (x, y) | Launches | Average us |", "|---|---|---:|---:|"]
    for (name, shape), v in sorted(by_shape.items(), key=lambda kv: (kv[0][0], -kv[0][1][0])):
        if "fmmprec" not in name or len(v) < 2 and sum(v) < 100:
            continue
        out.append("| `%s` | %d, %d | %d | %.2f |" % (name, shape[0], shape[1], len(v), sum(v) / len(v)))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", action="store_true",
                    help="counter-collection mode: one 512 MiB elementwise y = x*1 (the "
                         "calibration kernel of known size: 512 MiB read, 512 MiB written), "
                         "then 3 FMM applies, 3 preconditioner applies and one solve")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32", "split_fp16", "split_bf16"),
                    help="with --probe: the arithmetic of the probed plan")
    ap.add_argument("--theta", type=float, default=0.0,
                    help="with --probe: the MAC theta of the probed plan (0: list rule)")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="print markdown tables of a rocprofv3 kernel trace and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1308_3339_amd as fp
    from paper_1308_3339_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n, p = args.n, args.p
    N = n * n
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    f_host = inputs.gaussian_bumps(n, 16, seed=inputs.SEED_BUMPS_2048)
    f = torch.from_numpy(f_host).to(dev)
    u = torch.zeros(N, dtype=torch.float64, device=dev)

    log("setup n=%d p=%d" % (n, p))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    precs = {"fp64": fp.FMM_FP64, "fp32": fp.FMM_FP32, "split_fp16": fp.FMM_SPLIT_FP16,
             "split_bf16": fp.FMM_SPLIT_BF16}
    if (args.prec != "fp64" or args.theta != 0.0) and not args.probe:
        print("--prec and --theta apply to --probe only: the benchmark solve is the FP64 "
              "list-rule plan", file=sys.stderr)
        sys.exit(2)
    plan = fp.fmm_setup(n=n, p=p, bem=1, prec=precs[args.prec], theta=args.theta)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log("setup %.3f s" % setup_s)
    vec_blocks = plan.tune()     # autotuned Krylov vector-kernel grid (part of setup)
    m2l_split = plan.tune_m2l()  # autotuned M2L tile shape (list shares per tile)
    log("tuned vector blocks %d, M2L split %d" % (vec_blocks, m2l_split))

    if args.probe:
        x = torch.ones(64 << 20, dtype=torch.float64, device=dev)   # 512 MiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.mul(x, 1.0, out=y)     # calibration: reads 512 MiB, writes 512 MiB
        torch.cuda.synchronize()
        q = torch.from_numpy(inputs.random_charges(N, seed=9)).to(dev)
        out = torch.empty_like(q)
        for _ in range(3):
            plan.apply(q, out)
        for _ in range(3):
            plan.precond_apply(q, out)
        info = plan.solve(f, u)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "done", "copy_bytes_each_way": x.numel() * 8, "n": n, "p": p,
                          "solve_iters": info["iters"], "vector_blocks": vec_blocks}))
        plan.close()
        return

    for w in range(args.warmup):
        u.zero_()
        info = plan.solve(f, u)
        log("warmup %d: iters %d true rel res %.3e" % (w, info["iters"], info["true_rel_res"]))

    # timed region: K solves; the leaf kernel is timed by HIP events on this stream
    plan.profile(("LEAF",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        u.zero_()
        infos.append(plan.solve(f, u))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    leaf_ms, leaf_launches = plan.profile_read().get("LEAF", (0.0, 0))
    plan.profile(())
    log("timed %d solves in %.4f s" % (args.steps, t_total))
    ms_per_step = 1000.0 * t_total / args.steps
    solves_per_s = args.steps / t_total

    # correctness of the last solve (true residual recomputed on the GPU)
    w = torch.empty_like(u)
    plan.stencil_apply(u, w)
    rel_res = float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f))

    # per-stage breakdown of one solve (separate, untimed)
    plan.profile(fp.STAGES)
    u.zero_()
    plan.solve(f, u)
    sprof = plan.profile_read()
    stages = {k: round(v[0], 4) for k, v in sprof.items()}
    stage_roof = stage_rooflines(n, p, sprof)
    plan.profile(())

    # bare FMM and preconditioner throughput (HIP events on the same stream)
    q = torch.from_numpy(inputs.random_charges(N, seed=9)).to(dev)
    out = torch.empty_like(q)
    reps = 10
    for _ in range(2):
        plan.apply(q, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.apply(q, out)
    e1.record(stream)
    e1.synchronize()
    fmm_ms = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        plan.precond_apply(q, out)
    e1.record(stream)
    e1.synchronize()
    pc_ms = e0.elapsed_time(e1) / reps
    log("fmm apply %.3f ms, precond apply %.3f ms" % (fmm_ms, pc_ms))

    src_hash = leaf_kernel_hash()
    leaf_avg_ms = leaf_ms / max(leaf_launches, 1)
    flops = leaf_kernel_flops(n, p)
    achieved = flops / (leaf_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 4),
                "traffic": traffic_from_profile(src_hash), "kernel": "k_leaf_grid<10>",
                "avg_launch_ms": round(leaf_avg_ms, 5), "launches": leaf_launches,
                "flops_per_launch": flops}

    iters = infos[-1]["iters"]

    # preconditioner stages on the right-hand side f (ring potential, boundary
    # density, output), kept per plan to set against the oracle's
    def stages_of(pl):
        zz, ph, sg = torch.empty_like(f), torch.empty(4 * n, dtype=torch.float64, device=dev), \
            torch.empty(4 * n, dtype=torch.float64, device=dev)
        pl.precond_stages(f, zz, ph, sg)
        torch.cuda.synchronize()
        return {"z": zz.cpu().numpy(), "phi": ph.cpu().numpy(), "sigma": sg.cpu().numpy()}

    gpu_stages = {"fp64": stages_of(plan)}
    gpu_solutions = {"fp64": u.cpu().numpy()}

    # precision variants: same solve and tolerance, reduced-precision P2P/P2M/M2L
    def variant_block(prec, desc, peak, mfma_per_flop, label):
        pl = fp.fmm_setup(n=n, p=p, bem=1, prec=prec)
        pl.tune()
        pl.tune_m2l()
        for _ in range(args.warmup):
            u.zero_()
            pl.solve(f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u.zero_()
            inf = pl.solve(f, u)
        torch.cuda.synchronize()
        tv = time.perf_counter() - t0
        pl.stencil_apply(u, w)
        relv = float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f))
        z64, zv = torch.empty_like(q), torch.empty_like(q)
        plan.precond_apply(q, z64)
        pl.precond_apply(q, zv)
        perr = float((zv - z64).abs().max() / z64.abs().max())
        gpu_stages[label] = stages_of(pl)
        gpu_solutions[label] = u.cpu().numpy()
        pl.profile(fp.STAGES)
        u.zero_()
        pl.solve(f, u)
        prof = pl.profile_read()
        pl.close()
        stg = {k: round(v[0], 4) for k, v in prof.items()}
        leaf_ms_v, leaf_n_v = prof.get("LEAF", (0.0, 0))
        avg = leaf_ms_v / max(leaf_n_v, 1)
        ach = flops / (avg * 1e-3) / 1e12
        # M2L: 8 p^2 algorithmic flops per translation; in FP32 on the vector
        # ALU (k_m2l<P, float>) for FP32 plans, on the 16-bit matrix cores
        # (k_m2l_mfma16, the same hi/lo products as the near field) for split plans
        m2l_ms_v, m2l_n_v = prof.get("M2L", (0.0, 0))
        m2l_avg = m2l_ms_v / max(m2l_n_v, 1)
        m2l_flops = 8.0 * p * p * m2l_translations((n // 8).bit_length() - 1)
        m2l_ach = m2l_flops / (m2l_avg * 1e-3) / 1e12 if m2l_avg > 0 else 0.0
        return {"prec": desc, "solves_per_s": round(args.steps / tv, 4),
                "ms_per_step": round(1000.0 * tv / args.steps, 4),
                "speedup_vs_fp64": round((args.steps / tv) / solves_per_s, 3),
                "iters": inf["iters"], "true_rel_res": relv,
                "precond_max_rel_diff_vs_fp64": perr, "stages_ms_per_solve": stg,
                "leaf_roofline": {"bound": "mfma", "kernel": "near field + P2M",
                                  "avg_launch_ms": round(avg, 5),
                                  "achieved": round(ach, 3), "unit": "TFLOP/s",
                                  "mfma_flops_per_algorithmic_flop": mfma_per_flop,
                                  "peak": peak, "frac": round(ach * mfma_per_flop / peak, 4)},
                "m2l_roofline": (
                    {"bound": "mfma", "kernel": "k_m2l_mfma16<P, %s>" % ("bf16" if "BF16" in label.upper() else "f16"),
                     "avg_call_ms": round(m2l_avg, 5), "achieved": round(m2l_ach, 3),
                     "unit": "TFLOP/s", "mfma_flops_per_algorithmic_flop": mfma_per_flop,
                     "peak": peak, "frac": round(m2l_ach * mfma_per_flop / peak, 4)}
                    if prec in (fp.FMM_SPLIT_FP16, fp.FMM_SPLIT_BF16) else
                    {"bound": "alu", "kernel": "k_m2l<P, float>",
                     "avg_call_ms": round(m2l_avg, 5), "achieved": round(m2l_ach, 3),
                     "unit": "TFLOP/s", "peak": PEAK_FP32_VALU_TFLOPS,
                     "frac": round(m2l_ach / PEAK_FP32_VALU_TFLOPS, 4),
                     # the library is built without packed FP32 instructions,
                     # which halves the vector FP32 rate it can issue
                     "peak_unpacked": PEAK_FP32_VALU_TFLOPS / 2,
                     "frac_unpacked": round(2 * m2l_ach / PEAK_FP32_VALU_TFLOPS, 4)})}

    def mac_block(p_t, theta, prec=fp.FMM_FP64):
        """MAC theta (Sec. 5.2): the 2048^2 solve with the dual tree
        traversal's near disk and lists, next to the list-rule plan.  With
        prec = FMM_FP32 the near field of the disk runs on the FP32 matrix
        cores and M2L in FP32 (the single-precision P2P of Sec. 7.1)."""
        pl = fp.fmm_setup(n=n, p=p_t, bem=1, theta=theta, prec=prec)
        pl.tune()
        pl.tune_m2l()
        for _ in range(args.warmup):
            u.zero_()
            pl.solve(f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u.zero_()
            inf = pl.solve(f, u)
        torch.cuda.synchronize()
        tv = time.perf_counter() - t0
        pl.stencil_apply(u, w)
        relv = float(torch.linalg.vector_norm(f - w) / torch.linalg.vector_norm(f))
        pl.profile(fp.STAGES)
        u.zero_()
        pl.solve(f, u)
        prof = pl.profile_read()
        pl.close()
        # volume potential against the p = 14 list-rule potential (about 1e-9)
        uv, ur = torch.empty_like(q), torch.empty_like(q)
        with fp.fmm_setup(n=n, p=p_t, bem=0, theta=theta, prec=prec) as pv:
            pv.apply(q, uv)
        with fp.fmm_setup(n=n, p=14, bem=0) as pr:
            pr.apply(q, ur)
        dv = float(torch.linalg.vector_norm(uv - ur) / torch.linalg.vector_norm(ur))
        # near disk of the theta and the algorithmic flops of the leaf kernel
        lim = 2.0 / (theta * theta)
        kk = int(math.floor(math.sqrt(lim)))
        nl = n // 8
        pairs = 0
        for b in range(-kk, kk + 1):
            for a in range(-kk, kk + 1):
                if a * a + b * b <= lim:
                    pairs += (nl - abs(a)) * (nl - abs(b)) * 4096
        flops_t = 2.0 * pairs + 4.0 * p_t * n * n
        leaf_ms_t, leaf_n_t = prof.get("LEAF", (0.0, 0))
        avg = leaf_ms_t / max(leaf_n_t, 1)
        ach = flops_t / (avg * 1e-3) / 1e12
        fp32 = prec == fp.FMM_FP32
        peak_t = 157.3 if fp32 else PEAK_FP64_VALU_TFLOPS
        return {"p": p_t, "theta": theta, "prec": "fp32" if fp32 else "fp64", "near_leaves": sum(
                    1 for b in range(-kk, kk + 1) for a in range(-kk, kk + 1) if a * a + b * b <= lim),
                "solves_per_s": round(args.steps / tv, 4),
                "ms_per_step": round(1000.0 * tv / args.steps, 4),
                "speedup_vs_list_rule_p10": round((args.steps / tv) / solves_per_s, 3),
                "iters": inf["iters"], "true_rel_res": relv,
                "volume_rel_l2_diff_vs_p14": dv,
                "stages_ms_per_solve": {k: round(v[0], 4) for k, v in prof.items()},
                "leaf_roofline": {"bound": "mfma" if fp32 else "alu",
                                  "kernel": "k_leaf_wide_mfma32" if fp32 else "k_leaf_wide",
                                  "pairs": pairs, "avg_launch_ms": round(avg, 5),
                                  "achieved": round(ach, 3), "unit": "TFLOP/s", "peak": peak_t,
                                  "frac": round(ach / peak_t, 4)}}

    log("point cloud, 1M points")
    points = points_block(fp, inputs, torch, args.steps, args.warmup)
    log("points fp64 %.1f Mpoints/s, fp32 %.1f Mpoints/s" % (points["fp64"]["mpoints_per_s"],
                                                            points["fp32"]["mpoints_per_s"]))
    log("mac theta")
    mac = mac_block(6, 0.4)
    log("mac theta p=6 theta=0.4: %.2f solves/s, %d iterations" % (mac["solves_per_s"],
                                                                   mac["iters"]))
    mac32 = mac_block(6, 0.4, fp.FMM_FP32)
    log("mac theta fp32: %.2f solves/s, %d iterations" % (mac32["solves_per_s"], mac32["iters"]))
    log("precision variants")
    variant = variant_block(fp.FMM_FP32, "P2P and P2M as FP32 MFMA contractions, M2L in FP32; "
                            "M2M, L2L, L2P, boundary, stencil, Arnoldi FP64", 157.3, 1, "fp32")
    variant16 = variant_block(fp.FMM_SPLIT_FP16, "P2P and P2M as FP16 hi+lo MFMA products "
                              "(hi*hi + hi*lo + lo*hi, FP32 accumulation), M2L as the same products of "
                              "the list translations on the matrix cores; M2M, L2L, "
                              "L2P, boundary, stencil, Arnoldi FP64", 2500.0, 3, "split_fp16")
    variantb16 = variant_block(fp.FMM_SPLIT_BF16, "P2P and P2M as BF16 hi+lo MFMA products "
                               "(hi*hi + hi*lo + lo*hi + lo*lo, FP32 accumulation), M2L as the same "
                               "products on the matrix cores; M2M, L2L, L2P, boundary, stencil, "
                               "Arnoldi FP64", 2500.0, 4,
                               "split_bf16")
    log("fp32 variant %.2f solves/s, split-fp16 %.2f, split-bf16 %.2f" % (
        variant["solves_per_s"], variant16["solves_per_s"], variantb16["solves_per_s"]))
    log("variable coefficient")
    varcoef = varcoef_block(fp, inputs, torch, plan, f, args.steps, args.warmup)
    log("variable coefficient %.2f solves/s, %d iterations" % (varcoef["solves_per_s"],
                                                              varcoef["iters"]))
    log("batched uneven solves")
    batched = batched_block(fp, inputs, torch, args.steps, args.warmup)
    log("batched %.1f instances/s (sequential %.1f)" % (batched["instances_per_s"],
                                                        batched["sequential_instances_per_s"]))
    batched16 = batched_block(fp, inputs, torch, args.steps, args.warmup, prec=fp.FMM_SPLIT_FP16)
    batched["split_fp16"] = {k: batched16[k] for k in ("instances_per_s", "batch_ms", "p50_ms",
                                                       "p99_ms", "all_converged", "iters_min_max")}
    log("batched split-fp16 %.1f instances/s" % batched16["instances_per_s"])
    log("adjoint (1024^2 gradients)")
    adjoint = adjoint_block(fp, inputs, torch, args.steps, args.warmup)
    log("adjoint %.2f gradients/s, fd err %.2e" % (adjoint["gradients_per_s"],
                                                   adjoint["centre_grad_rel_err_vs_central_fd"]))
    log("1024^2 p sweep")
    psweep = psweep_block(fp, inputs, torch, args.steps, args.warmup)
    cpu = None
    if not args.no_cpu_baseline:
        import numpy as np
        log("cpu baseline (oracle solve) ...")
        cpu, ref = cpu_baseline(n, p, f_host)
        log("cpu baseline: setup %.2f s, solve %.2f s" % (cpu["setup_s"], cpu["solve_s"]))
        # every plan's preconditioner stages on f and its solution against the oracle's
        relmax = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
        for key, blk in (("fp64", None), ("fp32", variant), ("split_fp16", variant16),
                         ("split_bf16", variantb16)):
            g = gpu_stages[key]
            err = {"phi_ring": relmax(g["phi"], ref["phi"]), "sigma": relmax(g["sigma"], ref["sigma"]),
                   "z": relmax(g["z"], ref["z"]),
                   "solution_rel_l2": float(np.linalg.norm(gpu_solutions[key] - ref["x"])
                                            / np.linalg.norm(ref["x"]))}
            if blk is None:
                stage_err_fp64 = err
            else:
                blk["stage_rel_err_vs_fp64_oracle"] = err

    res = {
        "metric": "FMM-precond GMRES solves/s to 1e-8 rel. residual, 2048^2 grid; FMM Mpoints/s",
        "value": round(solves_per_s, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "5-point FD Poisson, %dx%d interior grid, zero Dirichlet data, "
                               "f = 16 Gaussian bumps (seed %d), FMM-BEM preconditioner p=%d "
                               "leaf 64, FGMRES(30) to 1e-8, FP64"
                               % (n, n, inputs.SEED_BUMPS_2048, p),
                   "n": n, "N": N, "p": p, "restart": 30, "tol": 1e-8},
        "fmm_mpoints_per_s": round(N / (fmm_ms * 1e-3) / 1e6, 2),
        "precond_mpoints_per_s": round(N / (pc_ms * 1e-3) / 1e6, 2),
        "fmm_apply_ms": round(fmm_ms, 4),
        "precond_apply_ms": round(pc_ms, 4),
        "iters": iters,
        "true_rel_res": rel_res,
        "setup_s": round(setup_s, 3),
        "tuned_vector_blocks": vec_blocks,
        "tuned_m2l_split": m2l_split,
        "stages_ms_per_solve": stages,
        "stage_rooflines": stage_roof,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stage_rel_err_vs_fp64_oracle": stage_err_fp64 if cpu else None,
        "p_sweep_1024": psweep,
        "variant_fp32": variant,
        "variant_split_fp16": variant16,
        "variant_split_bf16": variantb16,
        "adjoint": adjoint,
        "variable_coefficient": varcoef,
        "batched": batched,
        "mac_theta": mac,
        "mac_theta_fp32": mac32,
        "points": points,
    }
    plan.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
