"""Pins for the CPU FP64 oracle: closed forms, exact identities, invariances,
brute force and the paper's qualitative results.  No GPU involved.

Each test names the passage of arXiv:1308.3339 it pins.  A plausible mistake
in the oracle (a dropped term, a wrong sign or index, a transposed operand)
breaks at least one of these.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as o

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- direct sum
def test_direct_single_charge_closed_form():
    """Sec. 4.2 / 5.3: G(r) = -(1/2pi) log r for one unit charge."""
    tx = np.array([0.3, 1.7, -2.0, 0.5])
    ty = np.array([0.4, -0.2, 5.0, 0.5])
    u = o.direct([0.5], [0.5], [1.0], tx, ty, self_log=math.log(0.01))
    for t in range(4):
        r = math.hypot(tx[t] - 0.5, ty[t] - 0.5)
        want = -math.log(0.01) / (2 * math.pi) if r == 0 else -math.log(r) / (2 * math.pi)
        assert abs(u[t] - want) <= 1e-15 * max(1.0, abs(want))


def test_direct_linear_and_symmetric():
    """The sum is linear in q and the kernel is symmetric: q1.G q2 = q2.G q1."""
    n = 16
    rng = _rng(1)
    q1, q2 = rng.uniform(-1, 1, n * n), rng.uniform(-1, 1, n * n)
    u1, u2 = o.grid_direct(n, q1), o.grid_direct(n, q2)
    u12 = o.grid_direct(n, 2.0 * q1 - 3.0 * q2)
    assert np.allclose(u12, 2.0 * u1 - 3.0 * u2, rtol=0, atol=1e-13 * np.abs(u12).max())
    assert abs(q1 @ u2 - q2 @ u1) <= 1e-13 * abs(q1 @ u2)


@pytest.mark.parametrize("n", [16, 32, 64])
def test_direct_matches_fft_convolution(n):
    """Sec. 5.1 eq. volume_integral on the grid, two ways: O(N^2) loop in C and
    an FFT convolution with the kernel table in numpy."""
    q = _rng(n).uniform(-1, 1, n * n)
    ud, uf = o.grid_direct(n, q), o.grid_direct_fft(n, q)
    assert np.linalg.norm(ud - uf) <= 1e-13 * np.linalg.norm(ud)


# ---------------------------------------------------------------- operators
def test_p2m_then_m2m_equals_p2m_at_parent():
    """Sec. 5.3 items 1-2: shifting a truncated multipole is exact, so
    M2M(P2M about the child) == P2M about the parent, to rounding."""
    rng = _rng(2)
    p = 12
    child, parent = 0.25 + 0.25j, 0.5 + 0.5j
    x = 0.25 + rng.uniform(-0.1, 0.1, 40)
    y = 0.25 + rng.uniform(-0.1, 0.1, 40)
    q = rng.uniform(-1, 1, 40)
    Mc = o.p2m(p, child, x, y, q)
    Mp = o.m2m(Mc, child - parent)
    Md = o.p2m(p, parent, x, y, q)
    assert np.abs(Mp - Md).max() <= 1e-13 * np.abs(Md).max()


def test_multipole_evaluation_within_truncation_bound():
    """Sec. 5.3 item 1: the multipole series about the centre reproduces the
    far potential with the tail bound sum|q| (rho/R)^p / (p (1 - rho/R))."""
    rng = _rng(3)
    x, y, q = rng.uniform(-0.1, 0.1, 30), rng.uniform(-0.1, 0.1, 30), rng.uniform(-1, 1, 30)
    rho = np.hypot(x, y).max()
    for p in (4, 8, 12, 16):
        M = o.p2m(p, 0j, x, y, q)
        for w in (0.5 + 0.1j, -0.3 - 0.4j, 0.05 + 0.6j):
            exact = float(np.sum(q * np.log(np.abs(w - (x + 1j * y)))))
            R = abs(w)
            bound = np.abs(q).sum() * (rho / R) ** p / (p * (1 - rho / R))
            assert abs(o.m2p(M, w) - exact) <= bound + 1e-14


def test_m2l_matches_taylor_coefficients_of_a_point_source():
    """Sec. 5.3 item 3 against a closed form: for one unit charge at s the
    local coefficients of log(d + t - s) about t = 0 are
    L_0 = log(d - s), L_n = (-1)^(n+1) / (n (d - s)^n)."""
    p = 40
    for s, d in ((0.05 + 0.03j, 1.0 + 0.5j), (-0.04 + 0.06j, -0.7 + 0.9j)):
        M = o.p2m(p, 0j, [s.real], [s.imag], [1.0])
        L = o.m2l(M, d)
        assert abs(L[0].real - math.log(abs(d - s))) <= 1e-14
        for nn in range(1, 8):
            exact = (-1) ** (nn + 1) / (nn * (d - s) ** nn)
            assert abs(L[nn] - exact) <= 1e-12 * abs(exact)


def test_l2l_is_exact_recentring():
    """Sec. 5.3 items 4-5: L2P(L2L(L, c), t) == L2P(L, t + c)."""
    rng = _rng(4)
    p = 12
    Lp = rng.standard_normal(p) + 1j * rng.standard_normal(p)
    for c in (0.1 + 0.2j, -0.15 + 0.05j):
        Lc = o.l2l(Lp, c)
        for t in (0.03 - 0.04j, -0.1 + 0.07j):
            a, b = o.l2p(Lc, t), o.l2p(Lp, t + c)
            assert abs(a - b) <= 1e-13 * np.abs(Lp).sum()


def test_l2p_is_real_part_of_polynomial():
    """Sec. 5.3 item 5 on a hand-made expansion: L = (1, 2i, 3) at t = 1 + i
    gives Re(1 + 2i(1+i) + 3(1+i)^2) = Re(1 + 2i - 2 + 6i) = -1."""
    assert abs(o.l2p(np.array([1, 2j, 3]), 1 + 1j) - (-1.0)) <= 1e-15


# ---------------------------------------------------------------- lists
@pytest.mark.parametrize("L", [2, 3, 4])
def test_interaction_lists_cover_every_pair_once(L):
    """Sec. 5.2: near field (3x3 leaves) plus the M2L lists of the target leaf
    and its ancestors account for every source leaf exactly once."""
    nl = 1 << L
    for ty in range(nl):
        for tx in range(nl):
            cover = np.zeros((nl, nl), dtype=int)
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    if 0 <= tx + a < nl and 0 <= ty + b < nl:
                        cover[ty + b, tx + a] += 1
            for lev in range(2, L + 1):
                ax, ay = tx >> (L - lev), ty >> (L - lev)
                lst = o.m2l_list(lev, ax, ay)
                assert len(lst) <= 27
                w = 1 << (L - lev)
                for sx, sy in lst:
                    cover[sy * w:(sy + 1) * w, sx * w:(sx + 1) * w] += 1
            assert (cover == 1).all(), (tx, ty)


def test_interior_cell_has_27_list_entries():
    assert len(o.m2l_list(4, 7, 6)) == 27
    assert len(o.m2l_list(4, 0, 0)) == 12   # 4x4 children of the 2x2 parents, minus 2x2 adjacent


# ---------------------------------------------------------------- whole FMM
@pytest.mark.parametrize("n", [8, 16])
def test_fmm_without_far_field_equals_direct(n):
    """With L < 2 there is no M2L: the FMM is the direct sum (Sec. 5.1)."""
    q = _rng(n).uniform(-1, 1, n * n)
    uf, ud = o.grid_fmm(n, 6, q), o.grid_direct(n, q)
    assert np.abs(uf - ud).max() <= 1e-14 * np.abs(ud).max()


def test_fmm_error_decays_geometrically_in_p():
    """Sec. 5.3: accuracy is controlled by p.  Random charges (grids with
    smooth charges have symmetric cells whose error falls in steps)."""
    n = 64
    q = _rng(7).uniform(-1, 1, n * n)
    ue = o.grid_direct_fft(n, q)
    errs = []
    for p in (4, 6, 8, 10, 12, 14):
        uf = o.grid_fmm(n, p, q)
        errs.append(np.linalg.norm(uf - ue) / np.linalg.norm(ue))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 4.0
    assert errs[4] <= 1e-6          # p = 12
    assert errs[5] <= 1e-7          # p = 14


def test_fmm_ring_targets_match_direct():
    """Ring targets (attached to their boundary leaf) get the same accuracy."""
    n, p = 32, 12
    q = _rng(9).uniform(-1, 1, n * n)
    gx, gy = o.grid_points(n)
    rx, ry = o.ring_points(n)
    uf = o.grid_fmm(n, p, q, with_ring=True)[n * n:]
    ud = o.direct(gx, gy, q, rx, ry)
    assert np.linalg.norm(uf - ud) <= 1e-6 * np.linalg.norm(ud)


def _rot(Q):
    """(x, y) -> (1 - y, x): grid node (i, j) goes to (n-1-j, i)."""
    n = Q.shape[0]
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    R = np.empty_like(Q)
    R[I, n - 1 - J] = Q[J, I]
    return R


def test_fmm_rotation_covariance():
    """A 90-degree rotation of the charges about the square's centre rotates
    the FMM potential (the uniform tree, the lists and the truncated series
    are all covariant), ring values move one side along (s -> s+1)."""
    n, p = 32, 8
    Q = _rng(11).uniform(-1, 1, (n, n))
    u = o.grid_fmm(n, p, Q.reshape(-1), with_ring=True)
    ur = o.grid_fmm(n, p, _rot(Q).reshape(-1), with_ring=True)
    U, UR = u[:n * n].reshape(n, n), ur[:n * n].reshape(n, n)
    assert np.abs(_rot(U) - UR).max() <= 1e-13 * np.abs(U).max()
    ring, ringr = u[n * n:].reshape(4, n), ur[n * n:].reshape(4, n)
    assert np.abs(np.roll(ring, 1, axis=0) - ringr).max() <= 1e-13 * np.abs(ring).max()


def test_fmm_reflection_covariance():
    """x -> 1 - x reflects the FMM potential (conjugation of the series)."""
    n, p = 32, 8
    Q = _rng(12).uniform(-1, 1, (n, n))
    U = o.grid_fmm(n, p, Q.reshape(-1)).reshape(n, n)
    UF = o.grid_fmm(n, p, Q[:, ::-1].copy().reshape(-1)).reshape(n, n)
    assert np.abs(U[:, ::-1] - UF).max() <= 1e-13 * np.abs(U).max()


def test_points_fmm_against_direct():
    """Point-cloud form: uniform random points, i == j excluded, p = 12."""
    N = 8192
    rng = _rng(13)
    x, y, q = rng.uniform(0, 1, N), rng.uniform(0, 1, N), rng.uniform(-1, 1, N)
    L = math.ceil(math.log(N / 64, 4))
    uf = o.fmm(L, 0.0, 0.0, 1.0, 12, x, y, q, x, y, 0.0)
    ud = o.direct(x, y, q, x, y, 0.0)
    assert np.linalg.norm(uf - ud) <= 1e-6 * np.linalg.norm(ud)


# ---------------------------------------------------------------- stencil
@pytest.mark.parametrize("k,l", [(1, 1), (2, 5), (7, 3)])
def test_stencil_eigenfunctions(k, l):
    """A sin(k pi x) sin(l pi y) = (4/h^2)(sin^2(k pi h/2) + sin^2(l pi h/2)) * same."""
    n = 32
    h = o.grid_h(n)
    x, y = o.grid_points(n)
    v = np.sin(k * math.pi * x) * np.sin(l * math.pi * y)
    lam = 4 / h ** 2 * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
    assert np.abs(o.stencil(n, v) - lam * v).max() <= 1e-12 * lam


def test_stencil_symmetric_and_matches_kron():
    n = 16
    rng = _rng(14)
    u, v = rng.standard_normal(n * n), rng.standard_normal(n * n)
    assert abs(u @ o.stencil(n, v) - v @ o.stencil(n, u)) <= 1e-12 * abs(u @ o.stencil(n, v))
    assert np.abs(o.stencil(n, v) - o.stencil_matrix(n) @ v).max() <= 1e-10


# ---------------------------------------------------------------- BEM
def test_bem_self_panel_matches_quadrature():
    """Sec. 4.3: S_kk is the integral of G over its own element of length h."""
    from scipy.integrate import quad
    n = 16
    h = o.grid_h(n)
    S = o.bem_matrix(n)
    val, _ = quad(lambda t: -math.log(abs(t)) / (2 * math.pi), -h / 2, h / 2, points=[0.0])
    assert abs(S[0, 0] - val) <= 1e-12 * abs(val)


def test_bem_matrix_geometry():
    """S = S^T; off-diagonal entries h G(|y_k - y_l|) on the counter-clockwise ring."""
    n = 16
    h = o.grid_h(n)
    S = o.bem_matrix(n)
    assert np.abs(S - S.T).max() == 0.0
    # bottom node k=0 at (h, 0); right node k=0 at (1, h)
    d = math.hypot(1 - h, h)
    assert abs(S[0, n] - (-h * math.log(d) / (2 * math.pi))) <= 1e-15
    # bottom k=0 and top k=n-1, which sits at (h, 1): distance 1
    assert abs(S[0, 3 * n - 1]) <= 1e-16


def test_bem_lu_solve():
    n = 16
    S = o.bem_matrix(n)
    b = _rng(15).standard_normal(4 * n)
    LU = S.copy()
    piv = np.zeros(4 * n, dtype=np.int32)
    assert o.lib().orc_lu_factor(4 * n, o._ptr(LU), piv.ctypes.data_as(o._ip)) == 0
    x = b.copy()
    o.lib().orc_lu_solve(4 * n, o._ptr(LU), piv.ctypes.data_as(o._ip), o._ptr(x))
    assert np.abs(S @ x - b).max() <= 1e-12 * np.abs(b).max()


def test_preconditioner_exact_mode_matches_dense_numpy():
    """C preconditioner with exact sums == numpy dense P^{-1} built independently."""
    n = 16
    P = o.dense_preconditioner(n)
    r = _rng(16).standard_normal(n * n)
    pc = o.Preconditioner(n, exact=True)
    z, phi_ring, sigma = pc.apply(r, stages=True)
    assert np.abs(z - P @ r).max() <= 1e-13 * np.abs(P @ r).max()
    # collocation condition at the ring: S sigma = -phi_ring
    S = o.bem_matrix(n)
    assert np.abs(S @ sigma + phi_ring).max() <= 1e-12 * np.abs(phi_ring).max()


def test_preconditioner_fmm_close_to_exact():
    n = 64
    r = _rng(17).standard_normal(n * n)
    ze = o.Preconditioner(n, exact=True).apply(r)
    zf = o.Preconditioner(n, p=12).apply(r)
    assert np.linalg.norm(zf - ze) <= 1e-6 * np.linalg.norm(ze)


def test_preconditioner_solves_the_dirichlet_problem():
    """Sec. 4.1: volume potential + boundary correction approximates the
    Dirichlet solution operator; error vs u = sin(pi x) sin(pi y) falls with h
    (the paper reports first order for its BEM, Sec. 6.2)."""
    errs = []
    for n in (32, 64, 128):
        x, y = o.grid_points(n)
        u = np.sin(math.pi * x) * np.sin(math.pi * y)
        f = 2 * math.pi ** 2 * u
        z = o.Preconditioner(n, exact=True).apply(f)
        errs.append(np.linalg.norm(z - u) / np.linalg.norm(u))
    assert errs[0] < 0.01
    assert errs[1] < errs[0] / 1.6 and errs[2] < errs[1] / 1.6


def test_spectrum_bounded_like_table2():
    """Sec. 6.1 Table 2 pattern: kappa(P^-1 A) is O(1) and nearly constant in h,
    while without the boundary correction lambda_max grows with n."""
    gold = json.load(open(os.path.join(GOLD, "paper_table2_spectrum.json")))
    kap = []
    for n in (16, 32):
        P, A = o.dense_preconditioner(n), o.stencil_matrix(n)
        ev = np.linalg.eigvals(P @ A)
        assert np.abs(ev.imag).max() <= 1e-8
        kap.append(ev.real.max() / ev.real.min())
        ev0 = np.linalg.eigvals(o.dense_preconditioner(n, bem=False) @ A).real
        assert ev0.max() > 4.0 * ev.real.max()
    assert 1.0 < kap[0] < 2.0 * max(gold["kappa_PA"])
    assert abs(kap[1] - kap[0]) <= 0.05 * kap[0]


# ---------------------------------------------------------------- FGMRES
def test_manufactured_solution():
    """f = 2 pi^2 sin(pi x) sin(pi y) is an eigenvector of A, so the discrete
    solution is [(pi h/2)/sin(pi h/2)]^2 sin sin; its error against the
    continuous u is (pi h)^2/12 (1 + O(h^2)) = 1.94689e-4 at n = 64."""
    n = 64
    h = o.grid_h(n)
    x, y = o.grid_points(n)
    u = np.sin(math.pi * x) * np.sin(math.pi * y)
    uh = (math.pi * h / 2 / math.sin(math.pi * h / 2)) ** 2 * u
    pc = o.Preconditioner(n, p=10)
    xs, info = o.fgmres(n, 2 * math.pi ** 2 * u, pc)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
    assert np.linalg.norm(xs - uh) <= 1e-6 * np.linalg.norm(uh)
    e = np.linalg.norm(xs - u) / np.linalg.norm(u)
    assert abs(e - 1.94689e-4) <= 2e-3 * 1.94689e-4


def test_unpreconditioned_gmres_converges_in_one_step_on_eigenvector():
    n = 32
    x, y = o.grid_points(n)
    f = np.sin(math.pi * x) * np.sin(math.pi * y)
    _, info = o.fgmres(n, f, None)
    assert info["converged"] and info["iters"] == 1


def test_fgmres_matches_dense_solve():
    n = 16
    b = _rng(18).standard_normal(n * n)
    xe = np.linalg.solve(o.stencil_matrix(n), b)
    for pc in (None, o.Preconditioner(n, p=8)):
        xs, info = o.fgmres(n, b, pc, tol=1e-12, maxit=2000)
        assert info["converged"]
        assert np.linalg.norm(xs - xe) <= 1e-9 * np.linalg.norm(xe)


def test_fgmres_restart_and_warm_start():
    """Restarted runs (m = 5) converge to the same solution; a warm start at
    the solution returns with zero iterations."""
    n = 16
    b = _rng(19).standard_normal(n * n)
    pc = o.Preconditioner(n, p=8)
    x1, i1 = o.fgmres(n, b, pc, restart=5)
    x2, i2 = o.fgmres(n, b, pc, restart=30)
    assert i1["converged"] and i2["converged"]
    assert np.linalg.norm(x1 - x2) <= 1e-6 * np.linalg.norm(x2)
    x3, i3 = o.fgmres(n, b, pc, x0=x2)
    assert i3["iters"] == 0


def test_mesh_independent_iterations_like_table1():
    """Sec. 6.1 Table 1 pattern with the paper's source f = 1: iteration
    counts stay nearly constant as the mesh is refined."""
    gold = json.load(open(os.path.join(GOLD, "paper_table1_fmm_iterations.json")))
    its = []
    for n in (16, 32, 64, 128):
        pc = o.Preconditioner(n, p=10)
        _, info = o.fgmres(n, np.ones(n * n), pc)
        assert info["converged"]
        its.append(info["iters"])
    spread_paper = max(gold["fmm_iterations"]) - min(gold["fmm_iterations"])
    assert max(its) - min(its) <= spread_paper + 1
    assert max(its) <= 15


def test_gmres_residual_estimate_is_true_residual():
    """GMRES minimises ||b - A x_k|| over the Krylov space, and the Givens
    estimate |g_{k+1}| equals that true residual: stopping after k inner
    steps must report (nearly) the same value both ways, non-increasing in k."""
    n = 16
    b = _rng(20).standard_normal(n * n)
    pc = o.Preconditioner(n, p=8)
    prev = np.inf
    for k in range(1, 7):
        _, info = o.fgmres(n, b, pc, maxit=k, tol=1e-14)
        est, true = info["hist"][k - 1], info["true_rel_res"]
        assert abs(est - true) <= 1e-6 * true
        assert true <= prev * (1 + 1e-12)
        prev = true
