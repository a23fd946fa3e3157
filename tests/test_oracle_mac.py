"""Pins of the oracle's dual tree traversal with a MAC theta (Sec. 5.2), CPU only.

  * theta in (1/sqrt2, 1] gives back the Greengard-Rokhlin interaction lists
    of the pinned list oracle, and the FMM equals the list FMM to rounding;
  * for smaller theta the traversal's lists have a closed form on a uniform
    tree (a child pair failing the test implies its parents fail it, by the
    triangle inequality): the near set is the lattice disk |d|^2 <= 2/theta^2
    and the M2L list of a cell is the children of its parent's disk minus
    its own disk, with nothing at levels 0 and 1;
  * every pair of leaves is covered exactly once, by one P2P pair or by one
    M2L between ancestors;
  * accuracy: about six significant digits at p = 6, theta = 0.4 (the
    setting the paper's timing runs use), error falling as theta shrinks and
    as p grows, and a point cloud at p = 20 equal to the direct sum;
  * the preconditioner at p = 6, theta = 0.4 is within about six digits of
    the one with exact sums and converges as fast as the p = 10 list
    preconditioner.
"""
import math

import numpy as np
import pytest

import oracle as o
from paper_1308_3339_amd import inputs


def _group(m2l, level):
    d = {}
    for l, t, s in m2l:
        if l == level:
            d.setdefault(int(t), set()).add(int(s))
    return d


@pytest.mark.parametrize("theta", [0.75, 0.9, 1.0])
def test_gr_lists_for_large_theta(theta):
    L = 4
    m2l, p2p = o.dtt_lists(L, theta)
    assert not np.any(m2l[:, 0] < 2)
    for l in range(2, L + 1):
        nc = 1 << l
        got = _group(m2l, l)
        for iy in range(nc):
            for ix in range(nc):
                want = {sy * nc + sx for sx, sy in o.m2l_list(l, ix, iy)}
                assert got.get(iy * nc + ix, set()) == want, (l, ix, iy)
    nl = 1 << L
    near = {}
    for t, s in p2p:
        near.setdefault(int(t), set()).add(int(s))
    for iy in range(nl):
        for ix in range(nl):
            want = {(iy + b) * nl + ix + a for a in (-1, 0, 1) for b in (-1, 0, 1)
                    if 0 <= ix + a < nl and 0 <= iy + b < nl}
            assert near[iy * nl + ix] == want


def _disk(theta):
    lim = 2.0 / (theta * theta)
    k = int(math.floor(math.sqrt(lim))) + 1
    return {(a, b) for a in range(-k, k + 1) for b in range(-k, k + 1) if a * a + b * b <= lim}


@pytest.mark.parametrize("theta", [0.3, 0.4, 0.5, 0.6])
def test_closed_form_lists(theta):
    L = 5
    m2l, p2p = o.dtt_lists(L, theta)
    disk = _disk(theta)
    assert not np.any(m2l[:, 0] < 2)
    nl = 1 << L
    near = {}
    for t, s in p2p:
        near.setdefault(int(t), set()).add(int(s))
    for iy in range(nl):
        for ix in range(nl):
            want = {(iy + b) * nl + ix + a for a, b in disk if 0 <= ix + a < nl and 0 <= iy + b < nl}
            assert near[iy * nl + ix] == want
    for l in range(2, L + 1):
        nc = 1 << l
        got = _group(m2l, l)
        for iy in range(nc):
            for ix in range(nc):
                px, py = ix // 2, iy // 2
                want = set()
                for a, b in disk:
                    qx, qy = px + a, py + b
                    if not (0 <= qx < nc // 2 and 0 <= qy < nc // 2):
                        continue
                    for c in range(4):
                        sx, sy = 2 * qx + (c & 1), 2 * qy + (c >> 1)
                        if (sx - ix, sy - iy) not in disk:
                            want.add(sy * nc + sx)
                assert got.get(iy * nc + ix, set()) == want, (theta, l, ix, iy)


@pytest.mark.parametrize("theta", [0.3, 0.4, 0.55, 0.8])
def test_every_leaf_pair_covered_once(theta):
    L = 4
    nl = 1 << L
    m2l, p2p = o.dtt_lists(L, theta)
    cover = np.zeros((nl * nl, nl * nl), dtype=np.int32)
    cover[p2p[:, 0], p2p[:, 1]] += 1
    lx, ly = np.meshgrid(np.arange(nl), np.arange(nl), indexing="xy")
    lx, ly = lx.reshape(-1), ly.reshape(-1)
    for l, t, s in m2l:
        nc, sh = 1 << l, L - l
        tx, ty, sx, sy = t % nc, t // nc, s % nc, s // nc
        tm = ((lx >> sh) == tx) & ((ly >> sh) == ty)
        sm = ((lx >> sh) == sx) & ((ly >> sh) == sy)
        cover[np.ix_(tm, sm)] += 1
    assert cover.min() == 1 and cover.max() == 1


def test_large_theta_fmm_equals_list_fmm():
    n = 64
    q = inputs.gaussian_bumps(n, 16, seed=3) * o.grid_h(n) ** 2
    a = o.grid_fmm(n, 8, q, with_ring=True)
    b = o.grid_fmm(n, 8, q, with_ring=True, theta=0.8)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def _grid_err(n, p, theta):
    q = inputs.gaussian_bumps(n, 16, seed=3) * o.grid_h(n) ** 2
    ud = o.grid_direct_fft(n, q)
    u = o.grid_fmm(n, p, q, theta=theta)
    return np.linalg.norm(u - ud) / np.linalg.norm(ud)


def test_six_digits_at_p6_theta04_and_monotone():
    n = 64
    assert _grid_err(n, 6, 0.4) <= 1e-6
    for p in (4, 6, 8):
        e = [_grid_err(n, p, th) for th in (None, 0.6, 0.5, 0.4, 0.3)]
        assert all(b < a for a, b in zip(e, e[1:])), (p, e)
    e = [_grid_err(n, p, 0.4) for p in (4, 6, 8, 10)]
    assert all(b < a / 5 for a, b in zip(e, e[1:])), e


def test_point_cloud_high_order_equals_direct():
    rng = np.random.default_rng(11)
    N = 3000
    x, y = rng.random(N), rng.random(N)
    q = rng.standard_normal(N)
    ud = o.direct(x, y, q, x, y)
    for theta in (0.3, 0.5):
        u = o.fmm(3, 0.0, 0.0, 1.0, 20, x, y, q, x, y, theta=theta)
        assert np.abs(u - ud).max() <= 1e-10 * np.abs(ud).max()


def test_rejects_bad_theta():
    with pytest.raises(ValueError):
        o.dtt_lists(3, 0.0)
    with pytest.raises(ValueError):
        o.dtt_lists(3, 1.2)
    with pytest.raises(ValueError):
        o.Preconditioner(32, p=6, theta=1.5)


def test_preconditioner_accuracy_against_exact_sums():
    # both passes (volume and boundary sources) through the traversal: the
    # p = 6, theta = 0.4 operator is within about six digits of the one with
    # exact sums, where the p = 6 list operator is not
    n = 64
    r = inputs.gaussian_bumps(n, 16, seed=21)
    ze = o.Preconditioner(n, exact=True).apply(r)

    def err(**kw):
        z = o.Preconditioner(n, **kw).apply(r)
        return np.linalg.norm(z - ze) / np.linalg.norm(ze)
    assert err(p=6, theta=0.4) <= 2e-6
    assert err(p=6) >= 1e-5


def test_preconditioner_p6_theta04_iterations():
    n = 64
    f = inputs.gaussian_bumps(n, 16, seed=21)
    _, i10 = o.fgmres(n, f, o.Preconditioner(n, p=10))
    x6, i6 = o.fgmres(n, f, o.Preconditioner(n, p=6, theta=0.4))
    assert i6["converged"] and i6["true_rel_res"] <= 1e-8
    assert i6["iters"] <= i10["iters"] + 1
    _, igr = o.fgmres(n, f, o.Preconditioner(n, p=4))
    _, ith = o.fgmres(n, f, o.Preconditioner(n, p=4, theta=0.4))
    assert ith["iters"] <= igr["iters"]
