"""Oracle of the differentiation workload (numpy / scipy, FP64).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only the tests, the smoke
check and the benchmark's CPU-baseline leg use it, and it shares no code with
the HIP library.

The workload: L(f) = 0.5 |u - u_t|^2 with u = A^{-1} f, where A is the
5-point Dirichlet Laplacian of Sec. 2.1 (eq. axb) on the n x n interior grid,
and f is a sum of Gaussian bumps
    f_i = sum_k a_k exp(-|x_i - c_k|^2 / (2 w_k^2)).
Its gradients are
    dL/df = A^{-T} (u - u_t) = A^{-1} (u - u_t)          (A = A^T)
    dL/dc_k = sum_i (dL/df)_i a_k e_ik (x_i - c_k) / w_k^2,   e_ik = exp(...)
    dL/dw_k = sum_i (dL/df)_i a_k e_ik |x_i - c_k|^2 / w_k^3
    dL/da_k = sum_i (dL/df)_i e_ik.

Solves here are exact up to rounding: the sine transform (DST-I) diagonalises
A, with eigenvalues (4/h^2)(sin^2(j pi h/2) + sin^2(k pi h/2)) for the modes
sin(j pi x) sin(k pi y), j, k = 1..n (a closed form of the discrete
operator, not the paper's method).  Central differences of L built on this
solver are therefore free of Krylov tolerance noise.
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def grid_xy(n):
    """Interior nodes ((i+1)h, (j+1)h), row-major with x fastest, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(t, t, indexing="xy")
    return X.reshape(-1), Y.reshape(-1)


def fd_eigenvalues(n):
    """lambda_{jk} of A for the modes sin(j pi x) sin(k pi y), as an n x n
    array indexed [k-1, j-1] (y mode, x mode) to match the row-major grid."""
    h = 1.0 / (n + 1)
    s = np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    return (4.0 / (h * h)) * (s[:, None] + s[None, :])


def fd_solve_exact(n, b):
    """u = A^{-1} b for the 5-point Dirichlet Laplacian (zero ring data):
    DST-I in both directions, divide by the eigenvalues, inverse DST-I."""
    B = np.asarray(b, dtype=np.float64).reshape(n, n)
    U = scipy.fft.dstn(B, type=1) / fd_eigenvalues(n)
    return scipy.fft.idstn(U, type=1).reshape(-1)


def bumps_eval(n, cx, cy, w, a):
    """f_i = sum_k a_k exp(-|x_i - c_k|^2 / (2 w_k^2)) at the interior nodes."""
    x, y = grid_xy(n)
    f = np.zeros(n * n)
    for k in range(len(a)):
        r2 = (x - cx[k]) ** 2 + (y - cy[k]) ** 2
        f += a[k] * np.exp(-r2 / (2.0 * w[k] ** 2))
    return f


def bumps_grad(n, cx, cy, w, a, g):
    """Gradients of sum_i g_i f_i with respect to the bump parameters:
    returns (d/dcx, d/dcy, d/dw, d/da), each of length K."""
    x, y = grid_xy(n)
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    K = len(a)
    gcx, gcy, gw, ga = (np.zeros(K) for _ in range(4))
    for k in range(K):
        dx, dy = x - cx[k], y - cy[k]
        r2 = dx * dx + dy * dy
        e = np.exp(-r2 / (2.0 * w[k] ** 2))
        ge = g * e
        ga[k] = ge.sum()
        gcx[k] = a[k] * (ge * dx).sum() / w[k] ** 2
        gcy[k] = a[k] * (ge * dy).sum() / w[k] ** 2
        gw[k] = a[k] * (ge * r2).sum() / w[k] ** 3
    return gcx, gcy, gw, ga


def loss(n, f, u_t):
    """L = 0.5 |A^{-1} f - u_t|^2."""
    d = fd_solve_exact(n, f) - u_t
    return 0.5 * float(d @ d)


def loss_grad_f(n, f, u_t):
    """dL/df = A^{-T} (A^{-1} f - u_t); A^{-T} = A^{-1} since A is symmetric."""
    return fd_solve_exact(n, fd_solve_exact(n, f) - u_t)


def loss_diff(n, f_plus, f_minus, u_t):
    """L(f_plus) - L(f_minus), evaluated as (u+ - u-) . ((u+ + u-)/2 - u_t),
    which is the same number without subtracting two large sums."""
    up, um = fd_solve_exact(n, f_plus), fd_solve_exact(n, f_minus)
    return float((up - um) @ (0.5 * (up + um) - u_t))


def central_fd_f(n, f, u_t, idx, h=1e-6):
    """Central differences of L with respect to f at the given node indices."""
    out = np.zeros(len(idx))
    for m, i in enumerate(idx):
        fp, fm = f.copy(), f.copy()
        fp[i] += h
        fm[i] -= h
        out[m] = loss_diff(n, fp, fm, u_t) / (2.0 * h)
    return out


def central_fd_centres(n, cx, cy, w, a, u_t, h=1e-6):
    """Central differences of L(f(c)) with respect to every bump centre
    coordinate: returns (d/dcx, d/dcy)."""
    K = len(a)
    gx, gy = np.zeros(K), np.zeros(K)
    for k in range(K):
        for arr, out in ((cx, gx), (cy, gy)):
            cp, cm = arr.copy(), arr.copy()
            cp[k] += h
            cm[k] -= h
            if arr is cx:
                fp, fm = bumps_eval(n, cp, cy, w, a), bumps_eval(n, cm, cy, w, a)
            else:
                fp, fm = bumps_eval(n, cx, cp, w, a), bumps_eval(n, cx, cm, w, a)
            out[k] = loss_diff(n, fp, fm, u_t) / (2.0 * h)
    return gx, gy
