// C ABI of the gfx950 FMM-preconditioned Poisson solver: argument checks,
// plan setup (PCSetUp of Sec. 7.1 of arXiv:1308.3339) and the entry points.
// The operator tables, interaction lists and work lists are built on the
// host by host_setup.cpp (plain C++) and uploaded here.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <vector>

#include "fmm_internal.h"
#include "host_setup.h"

namespace fmmprec {

thread_local std::string g_setup_error;

int fail(fmm_plan *plan, int code, const std::string &msg)
{
    if (plan) plan->err = msg;
    else g_setup_error = msg;
    return code;
}

int m2l_kernel_setup(fmm_plan *pl);  // fmm_grid.hip

// layouts of the host-built tables and of the device vectors they fill
static_assert(sizeof(host::C2) == sizeof(double2) && sizeof(host::F2) == sizeof(float2) &&
                  sizeof(host::I4) == sizeof(int4) && sizeof(host::I4) == sizeof(M2LItem),
              "host table layouts");

template <class D, class T>
static int upload_as(fmm_plan *pl, D **dst, const std::vector<T> &src)
{
    static_assert(sizeof(D) == sizeof(T), "layout");
    FMM_HIP(pl, hipMalloc(dst, src.size() * sizeof(T)));
    FMM_HIP(pl, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return FMM_OK;
}

template <class T>
static int upload(fmm_plan *pl, T **dst, const std::vector<T> &src)
{
    return upload_as(pl, dst, src);
}

static int build_m2l_items(fmm_plan *pl);

static int build_tables(fmm_plan *pl)
{
    host::Tables t;
    std::string err;
    if (!host::build_tables(pl->p, pl->theta, pl->h, pl->self_eps, t, err)) return fail(pl, FMM_ERR_ARG, err);
    pl->nlist = t.nlist;
    int st;
    if ((st = upload(pl, &pl->tab.ktab32, t.kt32)) || (st = upload(pl, &pl->tab.p2m32, t.p2m32)) ||
        (st = upload(pl, &pl->tab.ktab16, t.kt16)) || (st = upload(pl, &pl->tab.p2m16, t.p2m16)) ||
        (st = upload(pl, &pl->tab.ktabb16, t.ktb16)) || (st = upload(pl, &pl->tab.p2mb16, t.p2mb16)) ||
        (st = upload_as(pl, &pl->tab.hank32, t.hank32)) || (st = upload_as(pl, &pl->tab.hankl, t.hankl)) ||
        (st = upload_as(pl, &pl->tab.hankl32, t.hankl32)) || (st = upload(pl, &pl->tab.rtab, t.rt)) ||
        (st = upload_as(pl, &pl->tab.m2m, t.m2m)) || (st = upload_as(pl, &pl->tab.l2l, t.l2l)) ||
        (st = upload_as(pl, &pl->tab.hank, t.hank)) || (st = upload_as(pl, &pl->tab.m2l_off, t.offs)) ||
        (st = upload(pl, &pl->tab.m2l_a, t.an)) || (st = upload(pl, &pl->tab.m2l_b, t.bk)) ||
        (st = upload_as(pl, &pl->tab.p2m, t.p2m)) || (st = upload_as(pl, &pl->tab.l2p, t.l2p)) ||
        (st = upload(pl, &pl->tab.ktab, t.kt)) || (st = upload(pl, &pl->tab.m2lt16, t.m2lt16)) ||
        (st = upload(pl, &pl->tab.m2ltb16, t.m2ltb16)))
        return st;
    return FMM_OK;
}

static int build_levels_and_work(fmm_plan *pl)
{
    host::Work w;
    const bool ring_lists = pl->kind == FMM_GRID && pl->bem;
    host::build_work(pl->L, pl->p, pl->K, pl->side, ring_lists, w);
    static_assert(host::kMaxLevelsH == kMaxLevels, "level table size");
    for (int l = 0; l <= kMaxLevels; ++l) {
        pl->lv.off[l] = w.off[l];
        pl->lv.logw[l] = w.logw[l];
    }
    pl->exp_elems = w.exp_elems;
    pl->m2l_tiles.resize(w.tiles.size());
    if (!w.tiles.empty()) std::memcpy(pl->m2l_tiles.data(), w.tiles.data(), w.tiles.size() * sizeof(M2LItem));
    int st;
    if ((st = build_m2l_items(pl)) != FMM_OK || (st = set_m2l_split(pl, default_m2l_split(pl))) != FMM_OK)
        return st;
    if (ring_lists && !w.ring.empty()) {
        pl->n_ring_cells = (int)w.ring.size();
        if ((st = upload_as(pl, &pl->ring_cells, w.ring))) return st;
        pl->n_ring_p2m = (int)w.ring_p2m.size();
        if ((st = upload_as(pl, &pl->ring_p2m_cells, w.ring_p2m))) return st;
    }
    return ensure_rhs(pl, 1);
}

RhsSet plan_rhs(const fmm_plan *pl, int64_t sv, const int *act)
{
    RhsSet rh;
    rh.sv = sv;
    rh.se = pl->exp_elems;
    rh.sr = 4 * pl->n;
    rh.sb = 3 * pl->n;
    rh.act = act;
    return rh;
}

int ensure_rhs(fmm_plan *pl, int nr)
{
    if (nr <= pl->rhs_cap) return FMM_OK;
    drop_step_graphs(pl);
    double2 **exps[] = {&pl->ws.M, &pl->ws.Lt, &pl->ws.Lm, &pl->ws.M2, &pl->ws.Lt2, &pl->ws.Lm2};
    for (double2 **e : exps)
        if (*e) {
            (void)hipFree(*e);
            *e = nullptr;
        }
    double **rings[] = {&pl->phi_ring, &pl->ring_q};
    for (double **r : rings)
        if (*r) {
            (void)hipFree(*r);
            *r = nullptr;
        }
    double2 **bhs[] = {&pl->bhat, &pl->shat};
    for (double2 **b : bhs)
        if (*b) {
            (void)hipFree(*b);
            *b = nullptr;
        }
    pl->rhs_cap = 0;
    if (pl->exp_elems > 0) {
        const size_t bytes = (size_t)pl->exp_elems * nr * sizeof(double2);
        if (hipMalloc(&pl->ws.M, bytes) != hipSuccess || hipMalloc(&pl->ws.Lt, bytes) != hipSuccess ||
            hipMalloc(&pl->ws.Lm, bytes * pl->m2l_split) != hipSuccess)
            return fail(pl, FMM_ERR_ALLOC, "expansion workspace allocation failed");
        pl->lm_parts = pl->m2l_split;
        pl->lm_part = pl->exp_elems * nr;
        if (pl->kind == FMM_GRID && pl->bem) {
            // the boundary-source pass writes only border tiles of M2 and only
            // the boundary band of Lm2: everything else must stay zero
            if (hipMalloc(&pl->ws.M2, bytes) != hipSuccess || hipMalloc(&pl->ws.Lt2, bytes) != hipSuccess ||
                hipMalloc(&pl->ws.Lm2, bytes) != hipSuccess)
                return fail(pl, FMM_ERR_ALLOC, "expansion workspace allocation failed");
            FMM_HIP(pl, hipMemset(pl->ws.M2, 0, bytes));
            FMM_HIP(pl, hipMemset(pl->ws.Lm2, 0, bytes));
        }
    }
    if (pl->kind == FMM_GRID) {
        const size_t n = (size_t)pl->n;
        if (hipMalloc(&pl->phi_ring, 4 * n * nr * sizeof(double)) != hipSuccess ||
            hipMalloc(&pl->ring_q, 4 * n * nr * sizeof(double)) != hipSuccess ||
            hipMalloc(&pl->bhat, 3 * n * nr * sizeof(double2)) != hipSuccess ||
            hipMalloc(&pl->shat, 3 * n * nr * sizeof(double2)) != hipSuccess)
            return fail(pl, FMM_ERR_ALLOC, "ring workspace allocation failed");
    }
    pl->rhs_cap = nr;
    return FMM_OK;
}

int default_m2l_split(const fmm_plan *pl)
{
    return host::default_m2l_split((int)pl->m2l_tiles.size(), pl->ncu);
}

int m2l_split_for(const fmm_plan *pl, int nr)
{
    int split = pl->m2l_split;
    for (int r = nr; r > 1 && split > 1; r >>= 1) split >>= 1;
    return split;
}

// the work items of every split
static int build_m2l_items(fmm_plan *pl)
{
    std::vector<host::I4> tiles(pl->m2l_tiles.size());
    if (!tiles.empty()) std::memcpy(tiles.data(), pl->m2l_tiles.data(), tiles.size() * sizeof(host::I4));
    for (int e = 0; e < 4; ++e) {
        const std::vector<host::I4> items = host::m2l_items(tiles, 1 << e);
        if (items.empty()) continue;
        const int st = upload_as(pl, &pl->m2l_items[e], items);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

int set_m2l_split(fmm_plan *pl, int split)
{
    if (split != 1 && split != 2 && split != 4 && split != 8)
        return fail(pl, FMM_ERR_ARG, "M2L split must be 1, 2, 4 or 8");
    drop_step_graphs(pl);
    if (pl->ws.Lm && split > pl->lm_parts) {
        (void)hipFree(pl->ws.Lm);
        pl->ws.Lm = nullptr;
        const size_t bytes = (size_t)pl->exp_elems * pl->rhs_cap * split * sizeof(double2);
        if (hipMalloc(&pl->ws.Lm, bytes) != hipSuccess)
            return fail(pl, FMM_ERR_ALLOC, "M2L sum workspace allocation failed");
        pl->lm_parts = split;
    }
    pl->m2l_split = split;
    return FMM_OK;
}

static void release(fmm_plan *pl)
{
    void *ptrs[] = {pl->tab.ktab32, pl->tab.p2m32, pl->tab.ktab16, pl->tab.p2m16, pl->tab.ktabb16,
                    pl->tab.p2mb16, pl->tab.hank32, pl->tab.hankl, pl->tab.hankl32, pl->tab.m2lt16, pl->tab.m2ltb16, pl->tab.m2m, pl->tab.l2l, pl->tab.hank, pl->tab.m2l_off, pl->tab.m2l_a, pl->tab.m2l_b,
                    pl->tab.p2m, pl->tab.l2p, pl->tab.ktab, pl->tab.rtab, pl->ws.M, pl->ws.Lt,
                    pl->ws.Lm, pl->ws.M2, pl->ws.Lt2, pl->ws.Lm2, pl->m2l_items[0], pl->m2l_items[1], pl->m2l_items[2], pl->m2l_items[3],
                    pl->ring_cells, pl->ring_p2m_cells, pl->X0, pl->X2, pl->X1, pl->Xh, pl->phi_ring, pl->ring_q,
                    pl->bhat, pl->shat, pl->perm, pl->leaf_start, pl->px, pl->py, pl->qs, pl->us,
                    pl->V, pl->Z, pl->w, pl->b, pl->partial, pl->dscal, pl->bump_part};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (pl->hpin) (void)hipHostFree(pl->hpin);
    drop_step_graphs(pl);
    release_group(pl);
    if (pl->bevent) (void)hipEventDestroy(pl->bevent);
    for (hipEvent_t e : pl->sevent)
        if (e) (void)hipEventDestroy(e);
    if (pl->bstream) (void)hipStreamDestroy(pl->bstream);
}


}  // namespace fmmprec

using namespace fmmprec;

extern "C" {

const char *fmm_version(void) { return "fmmprec 0.1 gfx950"; }

const char *fmm_last_error(const fmm_plan *plan)
{
    return plan ? plan->err.c_str() : g_setup_error.c_str();
}

int fmm_setup(const fmm_problem *prob, const fmm_params *prm, void *stream, fmm_plan **out)
{
    if (!out) return fail(nullptr, FMM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!prob || !prm) return fail(nullptr, FMM_ERR_ARG, "problem or params is NULL");
    if (prm->p < kPMin || prm->p > kPMax)
        return fail(nullptr, FMM_ERR_ARG, "p must be in [2, 20]");
    if (prm->leaf != 64) return fail(nullptr, FMM_ERR_ARG, "leaf must be 64");
    const bool split = prm->prec == FMM_SPLIT_FP16 || prm->prec == FMM_SPLIT_BF16;
    if (prm->prec != FMM_FP64 && prm->prec != FMM_FP32 && !split)
        return fail(nullptr, FMM_ERR_UNSUPPORTED,
                    "prec must be FMM_FP64, FMM_FP32, FMM_SPLIT_BF16 or FMM_SPLIT_FP16");
    if (split && prob->kind != FMM_GRID)
        return fail(nullptr, FMM_ERR_UNSUPPORTED, "split-precision plans are built for GRID plans");
    if (!(prm->self_eps >= 0.0) || !std::isfinite(prm->self_eps))
        return fail(nullptr, FMM_ERR_ARG, "self_eps must be finite and >= 0");
    if (!(prm->theta == 0.0 || (prm->theta >= kThetaMin && prm->theta <= 1.0)))
        return fail(nullptr, FMM_ERR_ARG, "theta must be 0 (interaction lists) or in [0.3, 1]");
    const int Kt = near_radius(prm->theta);
    if (Kt > 1 && (split || prm->p > kThetaPMax ||
                   (prm->prec == FMM_FP32 && prob->kind != FMM_GRID)))
        return fail(nullptr, FMM_ERR_UNSUPPORTED,
                    "theta < 1/sqrt(2) is built for FP64 plans and FP32 grid plans, with p <= 12");
    if (Kt > 1 && (int64_t)prm->p * (16 + 4 * Kt) * (16 + 4 * Kt) * 16 > kM2LMaxLds)
        return fail(nullptr, FMM_ERR_UNSUPPORTED, "p too large for this theta (M2L source tile exceeds LDS)");
    hipStream_t s = (hipStream_t)stream;
    fmm_plan *pl = new (std::nothrow) fmm_plan();
    if (!pl) return fail(nullptr, FMM_ERR_ALLOC, "host allocation failed");
    pl->kind = prob->kind;
    pl->n = prob->n;
    pl->p = prm->p;
    pl->prec = prm->prec;
    pl->bem = prm->bem ? 1 : 0;
    pl->set_theta(prm->theta);
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            ncu > 0)
            pl->ncu = ncu;
    }
    int st = FMM_OK;
    if (prob->kind == FMM_GRID) {
        const int64_t n = prob->n;
        int L = 0;
        while (((int64_t)8 << L) < n && L < 12) ++L;
        if (n < 8 || ((int64_t)8 << L) != n) {
            delete pl;
            return fail(nullptr, FMM_ERR_ARG, "GRID n must be 8 * 2^L with n <= 32768");
        }
        pl->L = L;
        pl->nl = 1 << L;
        pl->h = 1.0 / (double)(n + 1);
        pl->self_eps = prm->self_eps > 0.0 ? prm->self_eps
                                           : std::exp(-0.57721566490153286061) / (2.0 * std::sqrt(2.0));
        pl->x0 = pl->y0 = 0.5 * pl->h;
        pl->side = (double)n * pl->h;
    } else if (prob->kind == FMM_POINTS) {
        const int64_t N = prob->n;
        if (N < 1 || !prob->x || !prob->y || !(prob->side > 0.0) || !std::isfinite(prob->side) ||
            !std::isfinite(prob->x0) || !std::isfinite(prob->y0)) {
            delete pl;
            return fail(nullptr, FMM_ERR_ARG, "POINTS needs n >= 1, x, y and a root square with side > 0");
        }
        int L = 0;
        while (((int64_t)64 << (2 * L)) < N && L < 12) ++L;   // L = ceil(log4(N / 64))
        pl->L = L;
        pl->nl = 1 << L;
        pl->h = 1.0;                 // grid tables are unused by point clouds
        pl->self_eps = 1.0;
        pl->bem = 0;
        pl->x0 = prob->x0;
        pl->y0 = prob->y0;
        pl->side = prob->side;
    } else {
        delete pl;
        return fail(nullptr, FMM_ERR_ARG, "unknown problem kind");
    }
    if ((st = build_tables(pl)) || (st = build_levels_and_work(pl)) || (st = m2l_kernel_setup(pl))) {
        g_setup_error = pl->err;
        release(pl);
        delete pl;
        return st;
    }
    if (pl->kind == FMM_POINTS) {
        if ((st = points_setup(pl, prob->x, prob->y, s)) != FMM_OK) {
            g_setup_error = pl->err;
            release(pl);
            delete pl;
            return st;
        }
    }
    if (pl->kind == FMM_GRID && (st = bumps_scratch_init(pl)) != FMM_OK) {
        g_setup_error = pl->err;
        release(pl);
        delete pl;
        return st;
    }
    if (pl->kind == FMM_GRID && pl->bem) {
        if ((st = bem_setup(pl, s)) != FMM_OK) {
            g_setup_error = pl->err;
            release(pl);
            delete pl;
            return st;
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        g_setup_error = std::string("setup: ") + hipGetErrorString(e);
        release(pl);
        delete pl;
        return FMM_ERR_DEVICE;
    }
    *out = pl;
    return FMM_OK;
}

int fmm_profile(fmm_plan *pl, uint32_t mask)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (mask && pl->ev_pool.empty()) {
        const int pairs = 8192;
        pl->ev_pool.resize(2 * pairs);
        pl->ev_stage.assign(pairs, 0);
        for (auto &e : pl->ev_pool) FMM_HIP(pl, hipEventCreate(&e));
    }
    pl->prof_mask = mask;
    pl->ev_used = 0;
    return FMM_OK;
}

int fmm_profile_read(fmm_plan *pl, fmm_profile_stats *out)
{
    if (!pl || !out) return fail(pl, FMM_ERR_ARG, "plan or out is NULL");
    std::memset(out, 0, sizeof(*out));
    for (int i = 0; i < pl->ev_used; ++i) {
        FMM_HIP(pl, hipEventSynchronize(pl->ev_pool[2 * i + 1]));
        float ms = 0.0f;
        FMM_HIP(pl, hipEventElapsedTime(&ms, pl->ev_pool[2 * i], pl->ev_pool[2 * i + 1]));
        out->ms[pl->ev_stage[i]] += ms;
        out->launches[pl->ev_stage[i]] += 1;
    }
    return FMM_OK;
}

int fmm_destroy(fmm_plan *plan)
{
    if (!plan) return FMM_OK;
    (void)hipDeviceSynchronize();
    for (auto &e : plan->ev_pool) (void)hipEventDestroy(e);
    release(plan);
    delete plan;
    return FMM_OK;
}

int fmm_apply(fmm_plan *pl, const double *q, double *u, int nrhs, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (!q || !u || nrhs < 1) return fail(pl, FMM_ERR_ARG, "q/u NULL or nrhs < 1");
    if (q == u) return fail(pl, FMM_ERR_ARG, "u must not alias q");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (pl->kind == FMM_GRID) ? (size_t)pl->n * pl->n : (size_t)pl->n;
    if (pl->kind == FMM_GRID) {
        // the nrhs grids as one launch sequence, in chunks the workspace holds
        for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsChunk) {
            const int nr = std::min(kMaxRhsChunk, nrhs - r0);
            int st = ensure_rhs(pl, nr);
            if (st == FMM_OK)
                st = grid_volume_fmm(pl, q + r0 * N, 1.0, u + r0 * N, nullptr, false,
                                     plan_rhs(pl, (int64_t)N, nullptr), nr, s);
            if (st != FMM_OK) return st;
        }
        return FMM_OK;
    }
    for (int r = 0; r < nrhs; ++r) {
        int st = points_fmm(pl, q + r * N, u + r * N, s);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

int fmm_points_order(fmm_plan *pl, int32_t *perm, int32_t *leaf_start, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_POINTS) return fail(pl, FMM_ERR_ARG, "the point order needs a POINTS plan");
    if (!perm && !leaf_start) return fail(pl, FMM_ERR_ARG, "perm and leaf_start are both NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t nleaf = (size_t)pl->nl * pl->nl;
    if (perm)
        FMM_HIP(pl, hipMemcpyAsync(perm, pl->perm, (size_t)pl->n * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
    if (leaf_start)
        FMM_HIP(pl, hipMemcpyAsync(leaf_start, pl->leaf_start, (nleaf + 1) * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
    return FMM_OK;
}

int fmm_precond_apply(fmm_plan *pl, const double *r, double *z, int nrhs, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "preconditioner needs a GRID plan");
    if (!r || !z || nrhs < 1) return fail(pl, FMM_ERR_ARG, "r/z NULL or nrhs < 1");
    if (r == z) return fail(pl, FMM_ERR_ARG, "z must not alias r");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)pl->n * pl->n;
    if (nrhs == 1) return precond_apply_one(pl, r, z, nullptr, nullptr, s);
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsChunk) {
        const int nr = std::min(kMaxRhsChunk, nrhs - r0);
        int st = precond_apply_rhs(pl, r + r0 * N, z + r0 * N, nr, (int64_t)N, nullptr, s);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

int fmm_precond_stages(fmm_plan *pl, const double *r, double *z, double *phi_ring, double *sigma,
                       void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "preconditioner needs a GRID plan");
    if (!r || !z || r == z) return fail(pl, FMM_ERR_ARG, "r/z NULL or aliased");
    return precond_apply_one(pl, r, z, phi_ring, pl->bem ? sigma : nullptr, (hipStream_t)stream);
}

int fmm_stencil_apply(fmm_plan *pl, const double *v, double *w, int nrhs, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "stencil needs a GRID plan");
    if (!v || !w || nrhs < 1 || v == w) return fail(pl, FMM_ERR_ARG, "v/w NULL, aliased or nrhs < 1");
    return stencil_apply(pl, v, w, nrhs, (hipStream_t)stream);
}

int precond_gmres_solve(fmm_plan *pl, const double *f, const double *g, double *u,
                        const gmres_params *prm, gmres_result *res, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "solve needs a GRID plan");
    if (!f || !u) return fail(pl, FMM_ERR_ARG, "f or u is NULL");
    if (f == u) return fail(pl, FMM_ERR_ARG, "u must not alias f");
    gmres_params q{1e-8, 30, 600};
    if (prm) q = *prm;
    if (!(q.tol > 0.0) || !std::isfinite(q.tol)) return fail(pl, FMM_ERR_ARG, "tol must be > 0");
    if (q.restart < 1 || q.restart > 32) return fail(pl, FMM_ERR_ARG, "restart must be in [1, 32]");
    if (q.maxit < 1) return fail(pl, FMM_ERR_ARG, "maxit must be >= 1");
    return gmres_solve(pl, f, g, u, &q, res, (hipStream_t)stream);
}

int fmm_stencil_var_apply(fmm_plan *pl, const double *ax, const double *ay, const double *v,
                          double *w, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "stencil needs a GRID plan");
    if (!ax || !ay || !v || !w) return fail(pl, FMM_ERR_ARG, "ax, ay, v or w is NULL");
    if (v == w) return fail(pl, FMM_ERR_ARG, "w must not alias v");
    return stencil_var_apply(pl, ax, ay, v, w, (hipStream_t)stream);
}

int precond_gmres_solve_var(fmm_plan *pl, const double *ax, const double *ay, const double *f,
                            double *u, const gmres_params *prm, gmres_result *res, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "solve needs a GRID plan");
    if (!ax || !ay || !f || !u) return fail(pl, FMM_ERR_ARG, "ax, ay, f or u is NULL");
    if (f == u) return fail(pl, FMM_ERR_ARG, "u must not alias f");
    gmres_params q{1e-8, 30, 600};
    if (prm) q = *prm;
    if (!(q.tol > 0.0) || !std::isfinite(q.tol)) return fail(pl, FMM_ERR_ARG, "tol must be > 0");
    if (q.restart < 1 || q.restart > 32) return fail(pl, FMM_ERR_ARG, "restart must be in [1, 32]");
    if (q.maxit < 1) return fail(pl, FMM_ERR_ARG, "maxit must be >= 1");
    return gmres_solve(pl, f, nullptr, u, &q, res, (hipStream_t)stream, ax, ay);
}

int precond_gmres_solve_batch(fmm_plan *const *plans, int32_t count, const double *const *f,
                              double *const *u, const gmres_params *prm, gmres_result *res,
                              double *elapsed_ms, int32_t flags, void *stream)
{
    if (!plans || !f || !u) return fail(nullptr, FMM_ERR_ARG, "plans, f or u is NULL");
    if (count < 1 || count > 1024) return fail(nullptr, FMM_ERR_ARG, "count must be in [1, 1024]");
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return fail(nullptr, FMM_ERR_ARG, "a plan is NULL");
        plans[i]->err.clear();   // a failure leaves its message on the plan that failed
    }
    for (int i = 0; i < count; ++i) {
        fmm_plan *pl = plans[i];
        if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "batched solves need GRID plans");
        if (!f[i] || !u[i]) return fail(pl, FMM_ERR_ARG, "f[i] or u[i] is NULL");
        if (f[i] == u[i]) return fail(pl, FMM_ERR_ARG, "u[i] must not alias f[i]");
        for (int k = 0; k < i; ++k)
            if (plans[k] == pl) return fail(pl, FMM_ERR_ARG, "a plan appears twice in the batch");
    }
    if (flags & ~(FMM_BATCH_GRAPHS | FMM_BATCH_SEPARATE)) return fail(plans[0], FMM_ERR_ARG, "unknown flags");
    gmres_params q{1e-8, 30, 600};
    if (prm) q = *prm;
    if (!(q.tol > 0.0) || !std::isfinite(q.tol)) return fail(plans[0], FMM_ERR_ARG, "tol must be > 0");
    if (q.restart < 1 || q.restart > 32) return fail(plans[0], FMM_ERR_ARG, "restart must be in [1, 32]");
    if (q.maxit < 1) return fail(plans[0], FMM_ERR_ARG, "maxit must be >= 1");
    return gmres_solve_batch(plans, count, f, u, &q, res, elapsed_ms, (flags & FMM_BATCH_GRAPHS) != 0,
                             (flags & FMM_BATCH_SEPARATE) != 0,
                             (hipStream_t)stream);
}

int precond_gmres_solve_multi(fmm_plan *pl, int32_t nrhs, const double *f, double *u,
                              const gmres_params *prm, gmres_result *res, int32_t flags, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "solve needs a GRID plan");
    if (!f || !u || nrhs < 1) return fail(pl, FMM_ERR_ARG, "f or u is NULL, or nrhs < 1");
    if (f == u) return fail(pl, FMM_ERR_ARG, "u must not alias f");
    if (flags & ~FMM_BATCH_GRAPHS) return fail(pl, FMM_ERR_ARG, "unknown flags");
    gmres_params q{1e-8, 30, 600};
    if (prm) q = *prm;
    if (!(q.tol > 0.0) || !std::isfinite(q.tol)) return fail(pl, FMM_ERR_ARG, "tol must be > 0");
    if (q.restart < 1 || q.restart > 32) return fail(pl, FMM_ERR_ARG, "restart must be in [1, 32]");
    if (q.maxit < 1) return fail(pl, FMM_ERR_ARG, "maxit must be >= 1");
    const size_t N = (size_t)pl->n * pl->n;
    const bool graphs = (flags & FMM_BATCH_GRAPHS) && !pl->prof_mask;
    // the solve runs on the plan's own stream (graphs cannot be captured on
    // the null stream), ordered after the work on `stream`
    hipStream_t caller = (hipStream_t)stream;
    if (!pl->bstream) FMM_HIP(pl, hipStreamCreateWithFlags(&pl->bstream, hipStreamNonBlocking));
    if (!pl->bevent) FMM_HIP(pl, hipEventCreateWithFlags(&pl->bevent, hipEventDisableTiming));
    FMM_HIP(pl, hipEventRecord(pl->bevent, caller));
    FMM_HIP(pl, hipStreamWaitEvent(pl->bstream, pl->bevent, 0));
    int overall = FMM_OK;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsChunk) {
        const int nr = std::min(kMaxRhsChunk, nrhs - r0);
        std::vector<const double *> fp(nr);
        std::vector<double *> up(nr);
        for (int r = 0; r < nr; ++r) {
            fp[r] = f + (r0 + r) * N;
            up[r] = u + (r0 + r) * N;
        }
        const int st = gmres_solve_group(pl, nr, fp.data(), up.data(), &q, res ? res + r0 : nullptr,
                                         graphs, pl->bstream);
        if (st < 0) return st;
        if (st != FMM_OK) overall = st;
    }
    FMM_HIP(pl, hipEventRecord(pl->bevent, pl->bstream));
    FMM_HIP(pl, hipStreamWaitEvent(caller, pl->bevent, 0));
    FMM_HIP(pl, hipStreamSynchronize(caller));
    return overall;
}

int fmm_tune(fmm_plan *pl, void *stream, int32_t *vec_blocks)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "tuning needs a GRID plan");
    int chosen = 0;
    const int st = tune_vector_blocks(pl, (hipStream_t)stream, &chosen);
    if (st == FMM_OK && vec_blocks) *vec_blocks = chosen;
    return st;
}

int fmm_tune_m2l(fmm_plan *pl, void *stream, int32_t *split)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    int chosen = 0;
    const int st = tune_m2l_split(pl, (hipStream_t)stream, &chosen);
    if (st == FMM_OK && split) *split = chosen;
    return st;
}

int fmm_set_m2l_split(fmm_plan *pl, int32_t split)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (split != 1 && split != 2 && split != 4 && split != 8)
        return fail(pl, FMM_ERR_ARG, "M2L split must be 1, 2, 4 or 8");
    FMM_HIP(pl, hipDeviceSynchronize());
    return set_m2l_split(pl, split);
}

int fmm_get_m2l_split(const fmm_plan *pl, int32_t *split)
{
    if (!pl || !split) return FMM_ERR_ARG;
    *split = pl->m2l_split;
    return FMM_OK;
}

int precond_gmres_solve_adjoint(fmm_plan *pl, const double *g, double *lambda,
                                const gmres_params *prm, gmres_result *res, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (!g || !lambda) return fail(pl, FMM_ERR_ARG, "g or lambda is NULL");
    // A^T = A: the adjoint system is the forward one with zero ring data
    return precond_gmres_solve(pl, g, nullptr, lambda, prm, res, stream);
}

int fmm_bumps_eval(fmm_plan *pl, int32_t K, const double *cx, const double *cy, const double *w,
                   const double *a, double *f, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "bumps need a GRID plan");
    if (!cx || !cy || !w || !a || !f) return fail(pl, FMM_ERR_ARG, "NULL bump parameter or output");
    return bumps_eval(pl, K, cx, cy, w, a, f, (hipStream_t)stream);
}

int fmm_bumps_grad(fmm_plan *pl, int32_t K, const double *cx, const double *cy, const double *w,
                   const double *a, const double *g, double *gcx, double *gcy, double *gw,
                   double *ga, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "bumps need a GRID plan");
    if (!cx || !cy || !w || !a || !g) return fail(pl, FMM_ERR_ARG, "NULL bump parameter or g");
    return bumps_grad(pl, K, cx, cy, w, a, g, gcx, gcy, gw, ga, (hipStream_t)stream);
}

int fmm_bumps_grad_noalloc(fmm_plan *pl, int32_t K, const double *cx, const double *cy,
                           const double *w, const double *a, const double *g, double *gcx,
                           double *gcy, double *gw, double *ga, void *stream)
{
    if (!pl) return fail(nullptr, FMM_ERR_ARG, "plan is NULL");
    if (pl->kind != FMM_GRID) return fail(pl, FMM_ERR_ARG, "bumps need a GRID plan");
    if (!cx || !cy || !w || !a || !g) return fail(pl, FMM_ERR_ARG, "NULL bump parameter or g");
    return bumps_grad_noalloc(pl, K, cx, cy, w, a, g, gcx, gcy, gw, ga, (hipStream_t)stream);
}

}  // extern "C"
