"""Seeded synthetic workloads (numpy, FP64).  Shared by the tests, the bench
and the smoke check; holds none of the method's arithmetic.

Recipes:
  manufactured(n)        f = 2 pi^2 sin(pi x) sin(pi y) at the n x n nodes
  ones(n)                f = 1 (the paper's Sec. 6.1 source, sign flipped to -Lap u = 1)
  gaussian_bumps(n, K, seed)
      f(x) = sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2)); draws from
      numpy.random.default_rng(seed): centres (K x 2, U(0,1)), then widths
      (K, U(0.02, 0.1)), then amplitudes (K, U(-1, 1))
  bump_params(K, seed)   the (cx, cy, w, a) of those bumps
  random_points(N, seed_xy, seed_q)
      points U(0,1)^2 from default_rng(seed_xy) (x then y), charges
      U(-1, 1) from default_rng(seed_q)
  target_subset(N, m, seed)   m distinct indices drawn by default_rng(seed)
  var_faces(n, mu, mx, my)    face values of a = 1 + mu sin(mx pi X) sin(my pi Y),
      X = 2x - 1, Y = 2y - 1, for the variable-coefficient problem
"""
from __future__ import annotations

import math

import numpy as np

# seeds of the benchmark workloads
SEED_BUMPS_1024 = 1
SEED_POINTS_XY = 2
SEED_POINTS_Q = 3
SEED_POINTS_TARGETS = 4
SEED_BUMPS_2048 = 5
# differentiation workload (1024 x 1024): target source, source, FD coordinates
SEED_ADJ_TARGET = 6
SEED_ADJ_SOURCE = 7
SEED_ADJ_COORDS = 8


def grid_nodes(n):
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(t, t, indexing="xy")
    return X.reshape(-1), Y.reshape(-1)


def manufactured(n):
    x, y = grid_nodes(n)
    return 2.0 * math.pi ** 2 * np.sin(math.pi * x) * np.sin(math.pi * y)


def manufactured_solution(n):
    x, y = grid_nodes(n)
    return np.sin(math.pi * x) * np.sin(math.pi * y)


def ones(n):
    return np.ones(n * n)


def bump_params(K=16, seed=SEED_BUMPS_2048):
    """(cx, cy, w, a) of the K seeded bumps, drawn in the order above."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, (K, 2))
    w = rng.uniform(0.02, 0.1, K)
    a = rng.uniform(-1.0, 1.0, K)
    return c[:, 0].copy(), c[:, 1].copy(), w, a


def gaussian_bumps(n, K=16, seed=SEED_BUMPS_2048):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, (K, 2))
    w = rng.uniform(0.02, 0.1, K)
    a = rng.uniform(-1.0, 1.0, K)
    x, y = grid_nodes(n)
    f = np.zeros(n * n)
    for k in range(K):
        f += a[k] * np.exp(-((x - c[k, 0]) ** 2 + (y - c[k, 1]) ** 2) / (2.0 * w[k] ** 2))
    return f


def var_coefficient(x, y, mu, mx, my):
    """a = 1 + mu sin(mx pi X) sin(my pi Y) with X = 2x - 1, Y = 2y - 1 (the
    coefficient of the variable-coefficient problem, written in the
    coordinates of the square [-1, 1]^2 and mapped onto the unit square)."""
    return 1.0 + mu * np.sin(mx * math.pi * (2.0 * x - 1.0)) * np.sin(my * math.pi * (2.0 * y - 1.0))


def var_faces(n, mu, mx, my):
    """Face values of the coefficient for the 5-point flux stencil:
    ax[j, i] = a((i + 1/2) h, (j + 1) h), i = 0..n (n x (n+1), between nodes
    i-1 and i in x), ay[j, i] = a((i + 1) h, (j + 1/2) h), j = 0..n
    ((n+1) x n, between rows j-1 and j); h = 1/(n+1), flattened row-major."""
    h = 1.0 / (n + 1)
    xf = (np.arange(n + 1) + 0.5) * h
    xn = (np.arange(n) + 1.0) * h
    ax = var_coefficient(xf[None, :], xn[:, None], mu, mx, my)
    ay = var_coefficient(xn[None, :], xf[:, None], mu, mx, my)
    return ax.reshape(-1).copy(), ay.reshape(-1).copy()


def random_points(N, seed_xy=SEED_POINTS_XY, seed_q=SEED_POINTS_Q):
    r = np.random.default_rng(seed_xy)
    x = r.uniform(0.0, 1.0, N)
    y = r.uniform(0.0, 1.0, N)
    q = np.random.default_rng(seed_q).uniform(-1.0, 1.0, N)
    return x, y, q


def random_charges(N, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, N)


def target_subset(N, m, seed=SEED_POINTS_TARGETS):
    return np.sort(np.random.default_rng(seed).choice(N, size=min(m, N), replace=False))
