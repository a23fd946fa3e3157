"""ctypes binding of libfmmprec.so.  The functions keep the C names; Plan is a
thin owner of an fmm_plan*.  Device arrays are torch float64 CUDA tensors
(contiguous); the stream is torch's current stream unless one is given.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libfmmprec.so"

FMM_OK, FMM_NOT_CONVERGED = 0, 1
FMM_ERR_ARG, FMM_ERR_DEVICE, FMM_ERR_ALLOC, FMM_ERR_NUMERIC, FMM_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
FMM_GRID, FMM_POINTS = 0, 1
FMM_FP64, FMM_FP32, FMM_SPLIT_BF16, FMM_SPLIT_FP16 = 0, 1, 2, 3
FMM_BATCH_GRAPHS, FMM_BATCH_SEPARATE = 1, 2

# every symbol include/fmmprec.h declares
exported_symbols = (
    "fmm_setup", "fmm_apply", "fmm_precond_apply", "fmm_precond_stages", "fmm_stencil_apply",
    "precond_gmres_solve", "fmm_destroy", "fmm_last_error", "fmm_version", "fmm_profile",
    "fmm_profile_read", "precond_gmres_solve_adjoint", "fmm_bumps_eval", "fmm_bumps_grad",
    "fmm_stencil_var_apply", "precond_gmres_solve_var", "precond_gmres_solve_batch", "fmm_tune",
    "fmm_bumps_grad_noalloc", "fmm_points_order", "precond_gmres_solve_multi",
    "fmm_tune_m2l", "fmm_set_m2l_split", "fmm_get_m2l_split",
)

STAGES = ("P2M", "M2M", "M2L", "L2L", "LEAF", "RING", "BEM", "PASS2", "STENCIL", "ARNOLDI")


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fmmprec error %d: %s" % (code, msg))
        self.code = code


class fmm_problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("side", ctypes.c_double)]


class fmm_params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("leaf", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("bem", ctypes.c_int32), ("self_eps", ctypes.c_double),
                ("theta", ctypes.c_double)]


class gmres_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32)]


class fmm_profile_stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 16), ("launches", ctypes.c_int64 * 16)]


class gmres_result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("est_rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double)]


_lib = None


def library_path():
    return os.path.join(_PKG, _LIBNAME)


def load_library():
    """Load the in-tree libfmmprec.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise FmmError(FMM_ERR_DEVICE, "%s is not built (run paper_1308_3339_amd.build)" % path)
    L = ctypes.CDLL(path)
    vp, dp, i32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int
    L.fmm_setup.argtypes = [ctypes.POINTER(fmm_problem), ctypes.POINTER(fmm_params), vp,
                            ctypes.POINTER(vp)]
    L.fmm_setup.restype = i32
    L.fmm_apply.argtypes = [vp, dp, dp, i32, vp]
    L.fmm_apply.restype = i32
    L.fmm_precond_apply.argtypes = [vp, dp, dp, i32, vp]
    L.fmm_precond_apply.restype = i32
    L.fmm_precond_stages.argtypes = [vp, dp, dp, dp, dp, vp]
    L.fmm_precond_stages.restype = i32
    L.fmm_stencil_apply.argtypes = [vp, dp, dp, i32, vp]
    L.fmm_stencil_apply.restype = i32
    L.precond_gmres_solve.argtypes = [vp, dp, dp, dp, ctypes.POINTER(gmres_params),
                                      ctypes.POINTER(gmres_result), vp]
    L.precond_gmres_solve.restype = i32
    L.precond_gmres_solve_batch.argtypes = [vp, i32, vp, vp, ctypes.POINTER(gmres_params),
                                            ctypes.POINTER(gmres_result),
                                            ctypes.POINTER(ctypes.c_double), i32, vp]
    L.precond_gmres_solve_batch.restype = i32
    L.precond_gmres_solve_multi.argtypes = [vp, i32, dp, dp, ctypes.POINTER(gmres_params),
                                            ctypes.POINTER(gmres_result), i32, vp]
    L.precond_gmres_solve_multi.restype = i32
    L.fmm_tune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
    L.fmm_tune.restype = i32
    L.fmm_tune_m2l.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
    L.fmm_tune_m2l.restype = i32
    L.fmm_set_m2l_split.argtypes = [vp, i32]
    L.fmm_set_m2l_split.restype = i32
    L.fmm_get_m2l_split.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.fmm_get_m2l_split.restype = i32
    L.fmm_stencil_var_apply.argtypes = [vp, dp, dp, dp, dp, vp]
    L.fmm_stencil_var_apply.restype = i32
    L.precond_gmres_solve_var.argtypes = [vp, dp, dp, dp, dp, ctypes.POINTER(gmres_params),
                                          ctypes.POINTER(gmres_result), vp]
    L.precond_gmres_solve_var.restype = i32
    L.precond_gmres_solve_adjoint.argtypes = [vp, dp, dp, ctypes.POINTER(gmres_params),
                                              ctypes.POINTER(gmres_result), vp]
    L.precond_gmres_solve_adjoint.restype = i32
    L.fmm_bumps_eval.argtypes = [vp, i32, dp, dp, dp, dp, dp, vp]
    L.fmm_bumps_eval.restype = i32
    L.fmm_bumps_grad.argtypes = [vp, i32, dp, dp, dp, dp, dp, dp, dp, dp, dp, vp]
    L.fmm_bumps_grad.restype = i32
    L.fmm_bumps_grad_noalloc.argtypes = [vp, i32, dp, dp, dp, dp, dp, dp, dp, dp, dp, vp]
    L.fmm_bumps_grad_noalloc.restype = i32
    L.fmm_points_order.argtypes = [vp, vp, vp, vp]
    L.fmm_points_order.restype = i32
    L.fmm_destroy.argtypes = [vp]
    L.fmm_destroy.restype = i32
    L.fmm_last_error.argtypes = [vp]
    L.fmm_last_error.restype = ctypes.c_char_p
    L.fmm_version.argtypes = []
    L.fmm_version.restype = ctypes.c_char_p
    L.fmm_profile.argtypes = [vp, ctypes.c_uint32]
    L.fmm_profile.restype = i32
    L.fmm_profile_read.argtypes = [vp, ctypes.POINTER(fmm_profile_stats)]
    L.fmm_profile_read.restype = i32
    _lib = L
    return L


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, name, numel=None):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _iptr(t, name, numel):
    """Device pointer of a contiguous int32 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32:
        raise TypeError("%s must be an int32 CUDA tensor" % name)
    if not t.is_contiguous() or t.numel() < numel:
        raise ValueError("%s must be contiguous with >= %d elements" % (name, numel))
    return ctypes.c_void_p(t.data_ptr())


def _check(code, plan_ptr):
    if code < 0:
        msg = load_library().fmm_last_error(plan_ptr)
        raise FmmError(code, msg.decode() if msg else "")
    return code


def fmm_version():
    return load_library().fmm_version().decode()


def fmm_last_error(plan=None):
    p = plan._ptr if isinstance(plan, Plan) else plan
    return load_library().fmm_last_error(p).decode()


def fmm_setup(kind=FMM_GRID, n=64, p=10, bem=1, self_eps=0.0, x=None, y=None,
              x0=0.0, y0=0.0, side=1.0, leaf=64, prec=FMM_FP64, theta=0.0, stream=None):
    L = load_library()
    prob = fmm_problem(kind, n, None, None, x0, y0, side)
    if kind == FMM_POINTS:
        prob.x = _dptr(x, "x", n).value
        prob.y = _dptr(y, "y", n).value
    prm = fmm_params(p, leaf, prec, bem, self_eps, theta)
    out = ctypes.c_void_p()
    code = L.fmm_setup(ctypes.byref(prob), ctypes.byref(prm), _stream(stream), ctypes.byref(out))
    _check(code, None)
    return Plan(out, kind, n, p, bem)


def fmm_apply(plan, q, u, nrhs=1, stream=None):
    N = plan.npts
    code = load_library().fmm_apply(plan._ptr, _dptr(q, "q", N * nrhs), _dptr(u, "u", N * nrhs),
                                    nrhs, _stream(stream))
    return _check(code, plan._ptr)


def points_levels(N):
    """L = ceil(log4(N / 64)) of a POINTS plan with N points."""
    L = 0
    while (64 << (2 * L)) < N and L < 12:
        L += 1
    return L


def fmm_points_order(plan, perm=None, leaf_start=None, stream=None):
    """Copies the plan's tree order: perm (N int32) and leaf_start
    (4^L + 1 int32, leaves in Morton order)."""
    nleaf = 1 << (2 * points_levels(plan.n))
    code = load_library().fmm_points_order(plan._ptr, _iptr(perm, "perm", plan.n),
                                           _iptr(leaf_start, "leaf_start", nleaf + 1),
                                           _stream(stream))
    return _check(code, plan._ptr)


def fmm_precond_apply(plan, r, z, nrhs=1, stream=None):
    N = plan.npts
    code = load_library().fmm_precond_apply(plan._ptr, _dptr(r, "r", N * nrhs),
                                            _dptr(z, "z", N * nrhs), nrhs, _stream(stream))
    return _check(code, plan._ptr)


def fmm_precond_stages(plan, r, z, phi_ring=None, sigma=None, stream=None):
    N, m = plan.npts, 4 * plan.n
    code = load_library().fmm_precond_stages(plan._ptr, _dptr(r, "r", N), _dptr(z, "z", N),
                                             _dptr(phi_ring, "phi_ring", m),
                                             _dptr(sigma, "sigma", m), _stream(stream))
    return _check(code, plan._ptr)


def fmm_stencil_apply(plan, v, w, nrhs=1, stream=None):
    N = plan.npts
    code = load_library().fmm_stencil_apply(plan._ptr, _dptr(v, "v", N * nrhs),
                                            _dptr(w, "w", N * nrhs), nrhs, _stream(stream))
    return _check(code, plan._ptr)


def precond_gmres_solve(plan, f, u, g=None, tol=1e-8, restart=30, maxit=600, stream=None):
    N = plan.npts
    prm = gmres_params(tol, restart, maxit)
    res = gmres_result()
    code = load_library().precond_gmres_solve(plan._ptr, _dptr(f, "f", N),
                                              _dptr(g, "g", 4 * plan.n), _dptr(u, "u", N),
                                              ctypes.byref(prm), ctypes.byref(res),
                                              _stream(stream))
    _check(code, plan._ptr)
    return {"status": code, "converged": code == FMM_OK, "iters": res.iters,
            "restarts": res.restarts, "est_rel_res": res.est_rel_res,
            "true_rel_res": res.true_rel_res}


def precond_gmres_solve_multi(plan, f, u, nrhs, tol=1e-8, restart=30, maxit=600, graphs=True,
                              stream=None):
    """nrhs stacked right-hand sides on one plan (f, u: nrhs * n*n).  Returns
    {"status", "results": [per-instance dict]}."""
    N = plan.npts
    prm = gmres_params(tol, restart, maxit)
    res = (gmres_result * nrhs)()
    code = load_library().precond_gmres_solve_multi(plan._ptr, nrhs, _dptr(f, "f", N * nrhs),
                                                    _dptr(u, "u", N * nrhs), ctypes.byref(prm), res,
                                                    FMM_BATCH_GRAPHS if graphs else 0,
                                                    _stream(stream))
    _check(code, plan._ptr)
    return {"status": code,
            "results": [{"converged": r.true_rel_res <= tol, "iters": r.iters,
                         "restarts": r.restarts, "est_rel_res": r.est_rel_res,
                         "true_rel_res": r.true_rel_res} for r in res]}


def precond_gmres_solve_batch(plans, fs, us, tol=1e-8, restart=30, maxit=600, graphs=True,
                              stream=None, separate=False):
    """Solves A u_i = f_i on plans[i] for every i at once (distinct GRID plans).
    Returns {"status", "results": [per-instance dict], "elapsed_ms": [...]}."""
    count = len(plans)
    if not (len(fs) == len(us) == count):
        raise ValueError("plans, fs and us must have the same length")
    arr = ctypes.c_void_p * count
    P = arr(*[p._ptr.value for p in plans])
    F = arr(*[_dptr(f, "f", p.npts).value for f, p in zip(fs, plans)])
    U = arr(*[_dptr(u, "u", p.npts).value for u, p in zip(us, plans)])
    prm = gmres_params(tol, restart, maxit)
    res = (gmres_result * count)()
    el = (ctypes.c_double * count)()
    L = load_library()
    flags = (FMM_BATCH_GRAPHS if graphs else 0) | (FMM_BATCH_SEPARATE if separate else 0)
    code = L.precond_gmres_solve_batch(P, count, F, U, ctypes.byref(prm), res, el, flags,
                                       _stream(stream))
    if code < 0:
        msgs = [L.fmm_last_error(p._ptr) for p in plans] + [L.fmm_last_error(None)]
        msg = next((m.decode() for m in msgs if m), "")
        raise FmmError(code, msg)
    return {"status": code,
            "results": [{"converged": r.true_rel_res <= tol, "iters": r.iters,
                         "restarts": r.restarts, "est_rel_res": r.est_rel_res,
                         "true_rel_res": r.true_rel_res} for r in res],
            "elapsed_ms": list(el)}


def fmm_tune(plan, stream=None):
    """Autotunes the plan's Krylov vector-kernel block count; returns it."""
    out = ctypes.c_int32(0)
    _check(load_library().fmm_tune(plan._ptr, _stream(stream), ctypes.byref(out)), plan._ptr)
    return out.value


def fmm_tune_m2l(plan, stream=None):
    """Times the M2L list splits 1, 2, 4, 8 on the plan, keeps the fastest; returns it."""
    out = ctypes.c_int32(0)
    _check(load_library().fmm_tune_m2l(plan._ptr, _stream(stream), ctypes.byref(out)), plan._ptr)
    return out.value


def fmm_set_m2l_split(plan, split):
    """Sets the plan's M2L list split (1, 2, 4 or 8)."""
    return _check(load_library().fmm_set_m2l_split(plan._ptr, int(split)), plan._ptr)


def fmm_get_m2l_split(plan):
    """The plan's current M2L list split."""
    out = ctypes.c_int32(0)
    _check(load_library().fmm_get_m2l_split(plan._ptr, ctypes.byref(out)), plan._ptr)
    return out.value


def fmm_stencil_var_apply(plan, ax, ay, v, w, stream=None):
    """w = A v for the variable-coefficient flux stencil (face values ax, ay)."""
    n, N = plan.n, plan.npts
    code = load_library().fmm_stencil_var_apply(plan._ptr, _dptr(ax, "ax", n * (n + 1)),
                                                _dptr(ay, "ay", n * (n + 1)), _dptr(v, "v", N),
                                                _dptr(w, "w", N), _stream(stream))
    return _check(code, plan._ptr)


def precond_gmres_solve_var(plan, ax, ay, f, u, tol=1e-8, restart=30, maxit=600, stream=None):
    """Variable-coefficient solve, constant-coefficient FMM-BEM preconditioner."""
    n, N = plan.n, plan.npts
    prm = gmres_params(tol, restart, maxit)
    res = gmres_result()
    code = load_library().precond_gmres_solve_var(plan._ptr, _dptr(ax, "ax", n * (n + 1)),
                                                  _dptr(ay, "ay", n * (n + 1)), _dptr(f, "f", N),
                                                  _dptr(u, "u", N), ctypes.byref(prm),
                                                  ctypes.byref(res), _stream(stream))
    _check(code, plan._ptr)
    return {"status": code, "converged": code == FMM_OK, "iters": res.iters,
            "restarts": res.restarts, "est_rel_res": res.est_rel_res,
            "true_rel_res": res.true_rel_res}


def precond_gmres_solve_adjoint(plan, g, lam, tol=1e-8, restart=30, maxit=600, stream=None):
    """lambda = A^{-T} g (A^T = A); lam holds the initial guess on entry."""
    N = plan.npts
    prm = gmres_params(tol, restart, maxit)
    res = gmres_result()
    code = load_library().precond_gmres_solve_adjoint(plan._ptr, _dptr(g, "g", N),
                                                      _dptr(lam, "lam", N), ctypes.byref(prm),
                                                      ctypes.byref(res), _stream(stream))
    _check(code, plan._ptr)
    return {"status": code, "converged": code == FMM_OK, "iters": res.iters,
            "restarts": res.restarts, "est_rel_res": res.est_rel_res,
            "true_rel_res": res.true_rel_res}


def _bump_args(cx, cy, w, a):
    K = cx.numel()
    for t, nm in ((cy, "cy"), (w, "w"), (a, "a")):
        if t.numel() != K:
            raise ValueError("%s has %d elements, cx has %d" % (nm, t.numel(), K))
    return K, [_dptr(t, nm, K) for t, nm in ((cx, "cx"), (cy, "cy"), (w, "w"), (a, "a"))]


def fmm_bumps_eval(plan, cx, cy, w, a, f, stream=None):
    """f_i = sum_k a_k exp(-|x_i - c_k|^2 / (2 w_k^2)) on the plan's grid."""
    K, ptrs = _bump_args(cx, cy, w, a)
    code = load_library().fmm_bumps_eval(plan._ptr, K, *ptrs, _dptr(f, "f", plan.npts),
                                         _stream(stream))
    return _check(code, plan._ptr)


def fmm_bumps_grad(plan, cx, cy, w, a, g, gcx=None, gcy=None, gw=None, ga=None, stream=None):
    """Gradients of sum_i g_i f_i with respect to the bump parameters."""
    K, ptrs = _bump_args(cx, cy, w, a)
    outs = [_dptr(t, nm, K) for t, nm in ((gcx, "gcx"), (gcy, "gcy"), (gw, "gw"), (ga, "ga"))]
    code = load_library().fmm_bumps_grad(plan._ptr, K, *ptrs, _dptr(g, "g", plan.npts), *outs,
                                         _stream(stream))
    return _check(code, plan._ptr)


def fmm_bumps_grad_noalloc(plan, cx, cy, w, a, g, gcx=None, gcy=None, gw=None, ga=None,
                           stream=None):
    """fmm_bumps_grad without any device allocation (static workspace)."""
    K, ptrs = _bump_args(cx, cy, w, a)
    outs = [_dptr(t, nm, K) for t, nm in ((gcx, "gcx"), (gcy, "gcy"), (gw, "gw"), (ga, "ga"))]
    code = load_library().fmm_bumps_grad_noalloc(plan._ptr, K, *ptrs, _dptr(g, "g", plan.npts),
                                                 *outs, _stream(stream))
    return _check(code, plan._ptr)


def fmm_profile(plan, stages=()):
    """Enable hipEvent timing of the named stages (empty: disable)."""
    mask = 0
    for st in stages:
        mask |= 1 << STAGES.index(st)
    return _check(load_library().fmm_profile(plan._ptr, mask), plan._ptr)


def fmm_profile_read(plan):
    """{stage: (milliseconds, launches)} accumulated since fmm_profile."""
    out = fmm_profile_stats()
    _check(load_library().fmm_profile_read(plan._ptr, ctypes.byref(out)), plan._ptr)
    return {st: (out.ms[i], int(out.launches[i])) for i, st in enumerate(STAGES)
            if out.launches[i] > 0}


def fmm_destroy(plan):
    if isinstance(plan, Plan):
        plan.close()
        return FMM_OK
    return load_library().fmm_destroy(plan)


class Plan:
    """Owner of an fmm_plan*; methods mirror the C entry points."""

    def __init__(self, ptr, kind, n, p, bem):
        self._ptr = ptr
        self.kind, self.n, self.p, self.bem = kind, n, p, bem
        self.npts = n * n if kind == FMM_GRID else n

    apply = fmm_apply
    precond_apply = fmm_precond_apply
    precond_stages = fmm_precond_stages
    stencil_apply = fmm_stencil_apply
    solve = precond_gmres_solve
    solve_adjoint = precond_gmres_solve_adjoint
    solve_multi = precond_gmres_solve_multi
    stencil_var_apply = fmm_stencil_var_apply
    tune = fmm_tune
    tune_m2l = fmm_tune_m2l
    set_m2l_split = fmm_set_m2l_split
    m2l_split = property(fmm_get_m2l_split)
    solve_var = precond_gmres_solve_var
    bumps_eval = fmm_bumps_eval
    bumps_grad = fmm_bumps_grad
    bumps_grad_noalloc = fmm_bumps_grad_noalloc
    points_order = fmm_points_order
    profile = fmm_profile
    profile_read = fmm_profile_read

    def close(self):
        if self._ptr is not None and self._ptr.value:
            load_library().fmm_destroy(self._ptr)
        self._ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
