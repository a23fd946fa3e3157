"""Pins of the differentiation oracle (oracle/adjoint.py), CPU only.

Each piece is pinned to something other than itself:
  * the exact solve against a dense solve of the assembled 5-point matrix
    (brute force) and against the closed-form discrete solution of the
    manufactured problem;
  * the bump model's parameter gradients against central differences of the
    bump values;
  * the loss gradient (adjoint solve) and the chain to the bump centres
    against central differences of the loss.
"""
import math

import numpy as np
import pytest

import oracle as o
from oracle import adjoint as adj
from paper_1308_3339_amd import inputs


@pytest.mark.parametrize("n", [5, 8, 12])
def test_exact_solve_matches_dense_solve(n):
    b = np.random.default_rng(n).standard_normal(n * n)
    A = o.stencil_matrix(n)
    u = adj.fd_solve_exact(n, b)
    ud = np.linalg.solve(A, b)
    assert np.abs(u - ud).max() <= 1e-12 * np.abs(ud).max()


def test_exact_solve_manufactured_closed_form():
    # f = 2 pi^2 sin(pi x) sin(pi y) is an eigenvector of A; the discrete
    # solution is [(pi h/2) / sin(pi h/2)]^2 sin(pi x) sin(pi y)
    n = 64
    h = 1.0 / (n + 1)
    u = adj.fd_solve_exact(n, inputs.manufactured(n))
    c = ((math.pi * h / 2) / math.sin(math.pi * h / 2)) ** 2
    ue = c * inputs.manufactured_solution(n)
    assert np.abs(u - ue).max() <= 1e-13


def test_exact_solve_inverts_the_oracle_stencil():
    n = 40
    b = np.random.default_rng(3).standard_normal(n * n)
    r = o.stencil(n, adj.fd_solve_exact(n, b)) - b
    assert np.abs(r).max() <= 1e-9 * np.abs(b).max()


def test_bumps_eval_matches_input_generator():
    n = 33
    cx, cy, w, a = inputs.bump_params(16, seed=11)
    f = adj.bumps_eval(n, cx, cy, w, a)
    assert np.abs(f - inputs.gaussian_bumps(n, 16, seed=11)).max() <= 1e-14


def test_bumps_grad_against_central_differences():
    n = 24
    cx, cy, w, a = inputs.bump_params(5, seed=12)
    g = np.random.default_rng(13).standard_normal(n * n)
    gcx, gcy, gw, ga = adj.bumps_grad(n, cx, cy, w, a, g)
    hh = 1e-6
    for k in range(5):
        for arr, ref in ((cx, gcx), (cy, gcy), (w, gw), (a, ga)):
            p, m = arr.copy(), arr.copy()
            p[k] += hh
            m[k] -= hh
            args_p = [cx, cy, w, a]
            args_m = [cx, cy, w, a]
            i = [cx is arr, cy is arr, w is arr, a is arr].index(True)
            args_p[i], args_m[i] = p, m
            fd = (g @ adj.bumps_eval(n, *args_p) - g @ adj.bumps_eval(n, *args_m)) / (2 * hh)
            assert abs(ref[k] - fd) <= 1e-6 * max(abs(fd), 1e-3), (k, i)


def test_loss_gradient_against_central_differences():
    n = 32
    f = inputs.gaussian_bumps(n, 16, seed=21)
    u_t = adj.fd_solve_exact(n, inputs.gaussian_bumps(n, 8, seed=22))
    g = adj.loss_grad_f(n, f, u_t)
    idx = inputs.target_subset(n * n, 12, seed=23)
    fd = adj.central_fd_f(n, f, u_t, idx)
    err = np.abs(fd - g[idx]).max() / np.abs(g[idx]).max()
    assert err <= 1e-7
    # the loss difference formula equals L(f+) - L(f-) computed directly
    fp = f.copy()
    fp[idx[0]] += 1e-2
    assert abs(adj.loss_diff(n, fp, f, u_t) - (adj.loss(n, fp, u_t) - adj.loss(n, f, u_t))) \
        <= 1e-10 * adj.loss(n, f, u_t)


def test_centre_gradient_chain_against_central_differences():
    n = 32
    cx, cy, w, a = inputs.bump_params(6, seed=31)
    f = adj.bumps_eval(n, cx, cy, w, a)
    u_t = adj.fd_solve_exact(n, inputs.gaussian_bumps(n, 4, seed=32))
    lam = adj.loss_grad_f(n, f, u_t)
    gcx, gcy, _, _ = adj.bumps_grad(n, cx, cy, w, a, lam)
    fx, fy = adj.central_fd_centres(n, cx, cy, w, a, u_t)
    scale = max(np.abs(gcx).max(), np.abs(gcy).max())
    assert np.abs(gcx - fx).max() <= 1e-6 * scale
    assert np.abs(gcy - fy).max() <= 1e-6 * scale
