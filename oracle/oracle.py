"""Python face of the CPU FP64 oracle.

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use this module.  It shares no code with
the HIP library: it wraps ``fmm_oracle.c`` (plain C, FP64) through ctypes and
adds two numpy-only references that need no FMM at all:

* :func:`grid_direct_fft` -- the exact grid sum u = G q of Sec. 5.1
  (eq. volume_integral) as a zero-padded FFT convolution with the kernel table
  log(h |d|), self entry log(eps_s h);
* :func:`dense_preconditioner` -- P^{-1} = h^2 (G_OO - h G_OR S^{-1} G_RO) as
  a dense matrix, the boundary-corrected volume potential of Sec. 4.1 with
  every sum done exactly (for the spectral checks of Table 2).

Every array crossing into C is float64, C-contiguous.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB = os.path.join(_HERE, "libfmm_oracle.so")
# A prebuilt variant may be named here (used to confirm that the pins catch a
# deliberately planted mistake in a mutated copy of the oracle).
_LIB_OVERRIDE = os.environ.get("FMM_ORACLE_LIB")

# Self-term regularisation (reading of Sec. 4.2): G_self = -(1/2pi) log(eps_s h)
# with eps_s = exp(-gamma) / (2 sqrt 2), the constant that makes h^2 G match
# the 5-point lattice Green's function at short range.
EULER_GAMMA = 0.57721566490153286060651209008240243
EPS_SELF = math.exp(-EULER_GAMMA) / (2.0 * math.sqrt(2.0))

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile fmm_oracle.c into libfmm_oracle.so (gcc, -O3, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=gnu99", "-O3", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build()
            L = ctypes.CDLL(_LIB)
        L.orc_p2m.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                              _dp, _dp, _dp, _dp]
        L.orc_m2m.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_m2l.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_l2l.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_l2p.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double]
        L.orc_l2p.restype = ctypes.c_double
        L.orc_m2p.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double]
        L.orc_m2p.restype = ctypes.c_double
        L.orc_direct.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp, _dp,
                                 ctypes.c_double, _dp]
        L.orc_m2l_list.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip]
        L.orc_m2l_list.restype = ctypes.c_int
        L.orc_fmm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp, _dp,
                              ctypes.c_double, _dp]
        L.orc_fmm.restype = ctypes.c_int
        L.orc_fmm_theta.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    _dp, _dp, _dp, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
        L.orc_fmm_theta.restype = ctypes.c_int
        L.orc_dtt_lists.argtypes = [ctypes.c_int, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_int64), _ip, _ip]
        L.orc_dtt_lists.restype = ctypes.c_int
        L.orc_bucket_points.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                        _ip, _ip]
        L.orc_bucket_points.restype = ctypes.c_int
        L.orc_stencil.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_grid_points.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_ring_points.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_bem_matrix.argtypes = [ctypes.c_int, _dp]
        L.orc_lu_factor.argtypes = [ctypes.c_int, _dp, _ip]
        L.orc_lu_factor.restype = ctypes.c_int
        L.orc_lu_solve.argtypes = [ctypes.c_int, _dp, _ip, _dp]
        L.orc_pc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double]
        L.orc_pc_create.restype = ctypes.c_void_p
        L.orc_pc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_pc_apply.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_pc_apply_ex.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_pc_bem_solve.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_pc_bem_solve.restype = ctypes.c_int
        L.orc_fgmres.argtypes = [ctypes.c_int, ctypes.c_void_p, _dp, _dp, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, _ip, _dp, _dp]
        L.orc_fgmres.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


# --------------------------------------------------------------------------
# single operators (complex arrays of length p)
# --------------------------------------------------------------------------
def _to_pairs(z) -> np.ndarray:
    z = np.asarray(z, dtype=np.complex128)
    return _f64(np.stack([z.real, z.imag], axis=-1).reshape(-1))


def _from_pairs(a: np.ndarray) -> np.ndarray:
    return a[0::2] + 1j * a[1::2]


def p2m(p, centre, x, y, q):
    x, y, q = _f64(x), _f64(y), _f64(q)
    out = np.zeros(2 * p)
    lib().orc_p2m(p, centre.real, centre.imag, len(q), _ptr(x), _ptr(y), _ptr(q), _ptr(out))
    return _from_pairs(out)


def m2m(M, c):
    p = len(M)
    a, out = _to_pairs(M), np.zeros(2 * p)
    lib().orc_m2m(p, _ptr(a), c.real, c.imag, _ptr(out))
    return _from_pairs(out)


def m2l(M, d):
    p = len(M)
    a, out = _to_pairs(M), np.zeros(2 * p)
    lib().orc_m2l(p, _ptr(a), d.real, d.imag, _ptr(out))
    return _from_pairs(out)


def l2l(Lp, c):
    p = len(Lp)
    a, out = _to_pairs(Lp), np.zeros(2 * p)
    lib().orc_l2l(p, _ptr(a), c.real, c.imag, _ptr(out))
    return _from_pairs(out)


def l2p(Lc, t):
    a = _to_pairs(Lc)
    return lib().orc_l2p(len(Lc), _ptr(a), t.real, t.imag)


def m2p(M, w):
    a = _to_pairs(M)
    return lib().orc_m2p(len(M), _ptr(a), w.real, w.imag)


def m2l_list(level, ix, iy):
    out = np.zeros(54, dtype=np.int32)
    cnt = lib().orc_m2l_list(level, ix, iy, out.ctypes.data_as(_ip))
    return [(int(out[2 * a]), int(out[2 * a + 1])) for a in range(cnt)]


# --------------------------------------------------------------------------
# sums over point sets
# --------------------------------------------------------------------------
def direct(sx, sy, q, tx, ty, self_log=0.0):
    """u_t = -(1/2pi) sum_j q_j k(r_tj), k = log r, k(0) = self_log."""
    sx, sy, q, tx, ty = map(_f64, (sx, sy, q, tx, ty))
    u = np.zeros(len(tx))
    lib().orc_direct(len(q), _ptr(sx), _ptr(sy), _ptr(q), len(tx), _ptr(tx), _ptr(ty),
                     float(self_log), _ptr(u))
    return u


def fmm(L, x0, y0, side, p, sx, sy, q, tx, ty, self_log=0.0, theta=None):
    """FMM on a uniform tree; theta None: interaction lists (Sec. 5.2, GR
    rule), else the dual tree traversal with that MAC."""
    sx, sy, q, tx, ty = map(_f64, (sx, sy, q, tx, ty))
    u = np.zeros(len(tx))
    if theta is None:
        rc = lib().orc_fmm(L, x0, y0, side, p, len(q), _ptr(sx), _ptr(sy), _ptr(q), len(tx),
                           _ptr(tx), _ptr(ty), float(self_log), _ptr(u))
    else:
        rc = lib().orc_fmm_theta(L, x0, y0, side, p, float(theta), len(q), _ptr(sx), _ptr(sy),
                                 _ptr(q), len(tx), _ptr(tx), _ptr(ty), float(self_log), _ptr(u))
    if rc != 0:
        raise ValueError("orc_fmm rejected its arguments")
    return u


def bucket_points(L, x0, y0, side, x, y, morton=True):
    """Stable counting sort of the points by leaf (Sec. 5.1): returns
    (start, order) with start[k] the first sorted position of leaf key k
    (4^L + 1 entries; key = Morton index, or row-major ly 2^L + lx) and
    order[i] the original index of sorted position i."""
    x, y = _f64(x), _f64(y)
    start = np.zeros((1 << (2 * L)) + 1, dtype=np.int32)
    order = np.zeros(max(len(x), 1), dtype=np.int32)
    rc = lib().orc_bucket_points(L, float(x0), float(y0), float(side), 1 if morton else 0, len(x),
                                 _ptr(x), _ptr(y), start.ctypes.data_as(_ip),
                                 order.ctypes.data_as(_ip))
    if rc != 0:
        raise ValueError("orc_bucket_points rejected its arguments")
    return start, order[:len(x)]


def dtt_lists(L, theta):
    """Interaction pairs of the dual tree traversal (Sec. 5.2) on a uniform
    tree with L levels: (M2L triples (level, target cell, source cell),
    P2P pairs (target leaf, source leaf)), cells row-major."""
    cnt = (ctypes.c_int64 * 2)()
    if lib().orc_dtt_lists(L, float(theta), cnt, None, None) != 0:
        raise ValueError("orc_dtt_lists rejected its arguments")
    m2l = np.zeros(3 * cnt[0], dtype=np.int32)
    p2p = np.zeros(2 * cnt[1], dtype=np.int32)
    lib().orc_dtt_lists(L, float(theta), cnt, m2l.ctypes.data_as(_ip), p2p.ctypes.data_as(_ip))
    return m2l.reshape(-1, 3), p2p.reshape(-1, 2)


# --------------------------------------------------------------------------
# grid problem
# --------------------------------------------------------------------------
def grid_h(n):
    return 1.0 / (n + 1)


def grid_levels(n):
    L = 0
    while (8 << L) < n:
        L += 1
    if (8 << L) != n:
        raise ValueError("grid side must be 8 * 2^L")
    return L


def self_log(n, eps_s=EPS_SELF):
    return math.log(eps_s * grid_h(n))


def grid_points(n):
    x, y = np.zeros(n * n), np.zeros(n * n)
    lib().orc_grid_points(n, _ptr(x), _ptr(y))
    return x, y


def ring_points(n):
    x, y = np.zeros(4 * n), np.zeros(4 * n)
    lib().orc_ring_points(n, _ptr(x), _ptr(y))
    return x, y


def stencil(n, v):
    v = _f64(v).reshape(-1)
    w = np.zeros(n * n)
    lib().orc_stencil(n, _ptr(v), _ptr(w))
    return w


def grid_fmm(n, p, q, eps_s=EPS_SELF, with_ring=False, theta=None):
    """FMM volume potential of grid charges q at the interior nodes
    (and, with_ring, also at the 4n ring nodes appended at the end); theta
    selects the dual-tree-traversal interactions."""
    h, L = grid_h(n), grid_levels(n)
    gx, gy = grid_points(n)
    tx, ty = gx, gy
    if with_ring:
        rx, ry = ring_points(n)
        tx, ty = np.concatenate([gx, rx]), np.concatenate([gy, ry])
    return fmm(L, 0.5 * h, 0.5 * h, n * h, p, gx, gy, _f64(q).reshape(-1), tx, ty,
               self_log(n, eps_s), theta=theta)


def grid_direct(n, q, eps_s=EPS_SELF):
    gx, gy = grid_points(n)
    return direct(gx, gy, _f64(q).reshape(-1), gx, gy, self_log(n, eps_s))


def grid_direct_fft(n, q, eps_s=EPS_SELF):
    """Exact grid sum by FFT convolution: u = -(1/2pi) K * q with
    K(di, dj) = log(h sqrt(di^2 + dj^2)), K(0, 0) = log(eps_s h)."""
    h = grid_h(n)
    d = np.arange(-(n - 1), n)
    DI, DJ = np.meshgrid(d, d, indexing="xy")
    r2 = (DI.astype(np.float64) ** 2 + DJ.astype(np.float64) ** 2)
    with np.errstate(divide="ignore"):
        K = np.log(h * np.sqrt(r2))
    K[n - 1, n - 1] = math.log(eps_s * h)
    M = 2 * n - 1
    sz = 1
    while sz < M + n - 1:
        sz *= 2
    Q = np.fft.rfft2(_f64(q).reshape(n, n), s=(sz, sz))
    KK = np.fft.rfft2(K, s=(sz, sz))
    full = np.fft.irfft2(Q * KK, s=(sz, sz))
    u = full[n - 1:2 * n - 1, n - 1:2 * n - 1]
    return -u.reshape(-1) / (2.0 * math.pi)


def bem_matrix(n):
    S = np.zeros((4 * n, 4 * n))
    lib().orc_bem_matrix(n, _ptr(S))
    return S


class Preconditioner:
    """z = P^{-1} r: FMM (or exact sums) + boundary correction on an n x n grid."""

    def __init__(self, n, p=10, eps_s=EPS_SELF, bem=True, exact=False, theta=None):
        self.n = n
        self.h = grid_h(n)
        self._pc = lib().orc_pc_create(n, p, eps_s, int(bem), int(exact),
                                       0.0 if theta is None else float(theta))
        if not self._pc:
            raise ValueError("oracle preconditioner: bad arguments")

    def apply(self, r, stages=False):
        r = _f64(r).reshape(-1)
        z = np.zeros_like(r)
        if not stages:
            lib().orc_pc_apply(self._pc, _ptr(r), _ptr(z))
            return z
        phi_r, sig = np.zeros(4 * self.n), np.zeros(4 * self.n)
        lib().orc_pc_apply_ex(self._pc, _ptr(r), _ptr(z), _ptr(phi_r), _ptr(sig))
        return z, phi_r, sig

    def bem_solve(self, phi_ring):
        """sigma = -S^{-1} phi_ring with the preconditioner's factors of S."""
        phi = _f64(phi_ring).reshape(-1)
        sig = np.zeros_like(phi)
        if lib().orc_pc_bem_solve(self._pc, _ptr(phi), _ptr(sig)) != 0:
            raise ValueError("preconditioner was built without the boundary correction")
        return sig

    def close(self):
        if self._pc:
            lib().orc_pc_destroy(self._pc)
            self._pc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fgmres(n, b, pc=None, x0=None, tol=1e-8, restart=30, maxit=600):
    """Right-preconditioned FGMRES(restart); returns (x, info dict)."""
    b = _f64(b).reshape(-1)
    x = np.zeros_like(b) if x0 is None else _f64(x0).reshape(-1).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    st = lib().orc_fgmres(n, pc._pc if pc is not None else None, _ptr(b), _ptr(x), tol, restart,
                          maxit, ctypes.byref(it), ctypes.byref(rel), _ptr(hist))
    return x, {"converged": st == 0, "iters": it.value, "true_rel_res": rel.value,
               "hist": hist[:it.value].copy()}


def dense_preconditioner(n, eps_s=EPS_SELF, bem=True):
    """P^{-1} as a dense matrix with all sums exact (numpy only, small n)."""
    h = grid_h(n)
    gx, gy = grid_points(n)
    rx, ry = ring_points(n)
    dx = gx[:, None] - gx[None, :]
    dy = gy[:, None] - gy[None, :]
    r = np.hypot(dx, dy)
    np.fill_diagonal(r, 1.0)
    G = -np.log(r) / (2 * math.pi)
    np.fill_diagonal(G, -math.log(eps_s * h) / (2 * math.pi))
    P = G
    if bem:
        Gor = -np.log(np.hypot(gx[:, None] - rx[None, :], gy[:, None] - ry[None, :])) / (2 * math.pi)
        # collocation matrix of Sec. 4.3 built here in numpy (independent of the C one)
        S = -h * np.log(np.hypot(rx[:, None] - rx[None, :], ry[:, None] - ry[None, :])
                        + np.eye(4 * n)) / (2 * math.pi)
        np.fill_diagonal(S, -(h / (2 * math.pi)) * (math.log(h / 2) - 1.0))
        P = G - h * Gor @ np.linalg.solve(S, Gor.T)
    return h * h * P


def stencil_matrix(n):
    h = grid_h(n)
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    I = np.eye(n)
    return (np.kron(I, T) + np.kron(T, I)) / (h * h)
