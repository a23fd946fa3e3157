// Internal declarations of the gfx950 FMM-preconditioner library.
//
// Data layout in HBM (all FP64):
//   grid vectors      row-major n x n, node (i, j) at j*n + i
//   expansions        per level l (2..L) and coefficient k (0..p-1), a
//                     double2 (re, im) per cell: exp[off(l) + k*4^l + cell],
//                     cell = iy*2^l + ix.  Coefficient-major so that a wave
//                     reading coefficient k of 64 neighbouring cells is one
//                     contiguous 1 KB segment.
//   scaled expansions M~_k = M_k / w^k and L~_k = L_k w^k with w the cell
//                     width of the level, so every translation operator is
//                     level independent (only Re L_0 picks up M_0 log w).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "fmmprec.h"
#include "host_setup.h"

namespace fmmprec {

constexpr int kPMin = 2;
constexpr int kPMax = 20;
constexpr int kMaxLevels = 24;
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kInv2Pi = 1.0 / (2.0 * kPi);
constexpr double kLn2 = 0.693147180559945309417;
// MAC theta (Sec. 5.2): smallest accepted value (near radius K <= 4) and the
// LDS the M2L kernel may use for its source tile
constexpr double kThetaMin = 0.3;
constexpr int kMaxK = 4;
constexpr int kThetaPMax = 12;   // largest p built for theta < 1/sqrt(2)
constexpr int64_t kM2LMaxLds = 160 * 1024;
// right-hand sides one launch sequence takes at most (larger counts run in
// chunks of this many; each needs its own expansion workspace)
constexpr int kMaxRhsChunk = 16;

// Near radius in leaves of a MAC theta on the uniform tree: two cells of one
// level, radius r = w/sqrt2 each, are well separated when 2r < theta |d| w,
// i.e. |d|^2 > 2/theta^2; K is the largest k with (k, 0) not separated.
// theta = 0 selects the interaction lists of the list rule (K = 1).
inline int near_radius(double theta) { return host::near_radius(theta); }

// The right-hand sides of one launch, selected by blockIdx.z: the grid
// vectors of right-hand side r start r*sv doubles on, its expansions r*se
// double2, its ring arrays (4n) r*sr doubles and its boundary-solve products
// (3n) r*sb double2.  act (device, may be null) holds a nonzero flag for each
// right-hand side still to be computed; the blocks of the others return at
// once, so a captured launch sequence serves any subset of them.
struct RhsSet {
    int64_t sv = 0, se = 0, sr = 0, sb = 0;
    const int *act = nullptr;
};
__device__ __forceinline__ bool rhs_active(const RhsSet &rh, int r)
{
    return !rh.act || rh.act[r] != 0;
}

// Work item of the all-levels M2L launch: a tile of target cells at a level.
struct M2LItem {
    int32_t level;
    int32_t part;   // share of the interaction lists (0 .. m2l_split-1), and part of Workspace::Lm
    int32_t tx0, ty0;
};

// Per-level bookkeeping passed by value to kernels.
struct LevelInfo {
    int64_t off[kMaxLevels + 1];  // double2 offset of level l in an expansion buffer
    double logw[kMaxLevels + 1];  // log(cell width) at level l
};

// Device-resident FMM tables for one p.
struct FmmTables {
    double2 *m2m;     // [4 quadrants][p][p]  M~ parent = A_q M~ child (lower triangular)
    double2 *l2l;     // [4 quadrants][p][p]  L~ child = B_q L~ parent (upper triangular)
    double2 *hank;    // [7*7 offsets][2p-1]  Hankel generators of M2L (offset index (dy+3)*7+dx+3)
    int4 *m2l_off;    // [4 parity classes][27] (dx, dy, hank index, 0)
    double *m2l_a;    // [p]  (-1)^n / n!   M2L output scale
    double *m2l_b;    // [p]  input scale: -1 for k = 0, 1/(k-1)! for k >= 1
    double2 *p2m;     // [p][64] grid P2M weights, -tau_j^k / k (1 for k = 0)
    double2 *l2p;     // [64][p] grid L2P powers tau_j^k
    double *ktab;     // [31][31] log(h |d|), d in [-15, 15]^2, self entry log(eps h)
    double *rtab;     // [17][17] log(h |d|), |dx|, |dy| <= 16: ring node to interior node
    float *ktab32;    // FP32 copy of ktab (precision variant)
    float *p2m32;     // [16 ceil(2p/16)][64] P2M weights as real rows (2k: Re, 2k+1: Im), FP32
    _Float16 *ktab16; // [hi, lo][8 shifted copies][31 rows][40]: ktab split in two FP16 halves
    _Float16 *p2m16;  // [hi, lo][16 ceil(2p/16)][64]: p2m32 split in two FP16 halves
    __bf16 *ktabb16;  // as ktab16, split in two BF16 halves
    __bf16 *p2mb16;   // as p2m16, split in two BF16 halves
    float2 *hank32;   // FP32 copy of hank (precision variant)
    double2 *hankl;   // [4 parity classes][nlist][2p-1]: hank of each list entry, in list order
    float2 *hankl32;  // FP32 copy of hankl
    _Float16 *m2lt16; // matrix-core M2L operators of the list entries, FP16 hi then lo parts
    __bf16 *m2ltb16;  // the same as BF16 pairs
};

struct Workspace {
    double2 *M = nullptr;    // multipoles, levels 2..L
    double2 *Lt = nullptr;   // local expansions, levels 2..L
    double2 *Lm = nullptr;   // M2L sums, levels 2..L, in m2l_split parts lm_part apart
    // second (boundary-source) pass of the preconditioner
    double2 *M2 = nullptr;
    double2 *Lt2 = nullptr;
    double2 *Lm2 = nullptr;
};

}  // namespace fmmprec

struct fmm_plan {
    int kind = FMM_GRID;
    int64_t n = 0;        // GRID: side; POINTS: N
    int L = 0;            // leaf level
    int nl = 1;           // leaves per side, 2^L
    int p = 10;
    int prec = FMM_FP64;  // FMM_FP32: P2P and M2L in FP32
    int ncu = 256;        // compute units of the plan's device
    int bem = 1;
    // well-separatedness: theta = 0 is the list rule (3x3 near leaves);
    // otherwise the MAC of the dual tree traversal, whose near set on the
    // uniform tree is the lattice disk |d|^2 <= 2/theta^2 (radius K leaves,
    // kx[b] = largest |a| with (a, b) near), and nlist M2L offsets per cell
    double theta = 0.0;
    int K = 1;
    int kx[fmmprec::kMaxK + 1] = {1, 1, 1, 1, 1};
    int nlist = 27;
    bool in_near(int dx, int dy) const { return fmmprec::host::in_near(theta, dx, dy); }
    void set_theta(double t)
    {
        theta = t;
        K = fmmprec::near_radius(t);
        for (int b = 0; b <= fmmprec::kMaxK; ++b) {
            int a = -1;
            while (a + 1 <= K && in_near(a + 1, b)) ++a;
            kx[b] = a;   // -1: no near leaf at distance b
        }
    }
    double h = 0.0;       // GRID mesh width
    double self_eps = 0.0;
    double x0 = 0.0, y0 = 0.0, side = 1.0;  // tree root square
    fmmprec::LevelInfo lv{};
    int64_t exp_elems = 0;                  // double2 elements per expansion buffer
    // right-hand sides the workspace holds side by side (expansions, ring
    // potential, boundary-solve products, ring charges); one per plan at
    // setup, more when a call stacks several (ensure_rhs)
    int rhs_cap = 0;

    fmmprec::FmmTables tab{};
    fmmprec::Workspace ws{};
    // M2L work items for each split S = 1, 2, 4, 8 (entry log2 S): every tile
    // of levels 2..L, S times (one item per list share)
    fmmprec::M2LItem *m2l_items[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<fmmprec::M2LItem> m2l_tiles;  // the tiles themselves (host copy)
    int m2l_split = 1;        // M2L blocks per tile for one right-hand side
    int lm_parts = 0;         // parts Workspace::Lm holds (>= m2l_split once allocated)
    int64_t lm_part = 0;      // double2 elements between parts of Lm (rhs_cap * exp_elems)
    int4 *ring_cells = nullptr;   // strips within 2K+1 cells of the boundary (see k_m2l_ring)
    int n_ring_cells = 0;
    int4 *ring_p2m_cells = nullptr;  // boundary cells of levels 2..L: (level, ix, iy, 0)
    int n_ring_p2m = 0;

    // boundary correction (GRID, bem = 1): inverses of the three distinct
    // diagonal blocks of the rotation-diagonalised collocation matrix
    double *X0 = nullptr;     // n x n real
    double *X2 = nullptr;     // n x n real
    double2 *X1 = nullptr;    // n x n complex
    double *Xh = nullptr;     // the three folded into 8 even/odd halves of (n/2)^2 (setup frees X0, X2, X1)
    double *phi_ring = nullptr;   // 4n
    double *ring_q = nullptr;     // 4n  (h * sigma)
    double2 *bhat = nullptr;      // 3n  (b^_0, b^_2 real parts in .x; b^_1 complex)
    double2 *shat = nullptr;      // 3n

    // POINTS
    int *perm = nullptr;          // sorted position -> caller index
    int *leaf_start = nullptr;    // 4^L + 1
    double *px = nullptr, *py = nullptr;  // sorted coordinates
    double *qs = nullptr, *us = nullptr;  // sorted charges / potentials

    // Krylov workspace (GRID)
    int kry_m = 0;
    int64_t ldb = 0;      // element stride between Krylov basis vectors (n^2 plus padding)
    double *V = nullptr;          // (m+1) x N
    double *Z = nullptr;          // m x N
    double *w = nullptr, *b = nullptr;
    double *partial = nullptr;    // reduction partials
    double *dscal = nullptr;      // small device scalars / coefficient vectors
    double *hpin = nullptr;       // pinned host mirror of dscal (two slots)
    hipEvent_t sevent[2] = {nullptr, nullptr};   // end of step j's copy, slot j & 1

    // bump-gradient reduction partials (allocated on first use), and the
    // device address of the library's static workspace on the plan's device
    // (used by the allocation-free entry point; not owned by the plan)
    double *bump_part = nullptr;
    double *bump_scratch = nullptr;

    // Krylov vector kernels: tuned block count (0: one block per 1024 elements)
    int vec_blocks = 0;
    // batched solves: the plan's own stream and completion event, and the
    // captured Arnoldi steps (graph j replays step j on this plan's buffers)
    hipStream_t bstream = nullptr;
    hipEvent_t bevent = nullptr;
    std::vector<hipGraphExec_t> step_exec;

    // group solves (many right-hand sides of this plan's size at once,
    // krylov.hip): capacity g_cap instances with restart g_m
    int g_cap = 0, g_m = 0;
    int64_t g_vs = 0;             // doubles per instance in g_basis: V (m+1) then Z (m)
    double *g_basis = nullptr;
    double *g_b = nullptr, *g_x = nullptr, *g_w = nullptr;   // g_cap grids each
    double *g_part = nullptr, *g_dscal = nullptr;
    void *g_state = nullptr;      // per-instance solver state (device)
    int *g_flags = nullptr;       // [run | fin | status] per instance (device)
    int *g_host = nullptr;        // pinned mirror: run, then status per instance
    std::vector<hipGraphExec_t> g_step_exec;   // step j of a group solve
    hipGraphExec_t g_end_exec = nullptr;      // end of a cycle
    int g_graph_nr = 0;           // instance count, maxit and tol the graphs were captured for
    int g_graph_maxit = 0;        // (the restart length is fixed by g_m)
    double g_graph_tol = 0.0;

    // stage timing (fmm_profile)
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;          // created on first enable
    std::vector<int> ev_stage;                // stage of event pair i (events 2i, 2i+1)
    int ev_used = 0;

    std::string err;
};

namespace fmmprec {

// status helpers
int fail(fmm_plan *plan, int code, const std::string &msg);
extern thread_local std::string g_setup_error;

#define FMM_HIP(plan, call)                                                       \
    do {                                                                          \
        hipError_t e__ = (call);                                                  \
        if (e__ != hipSuccess)                                                    \
            return ::fmmprec::fail((plan), FMM_ERR_DEVICE,                        \
                                   std::string(#call ": ") + hipGetErrorString(e__)); \
    } while (0)

// Scoped hipEvent pair around the launches of one stage (no-op unless the
// stage is enabled by fmm_profile).
struct StageTimer {
    fmm_plan *pl;
    hipStream_t s;
    int pair = -1;
    StageTimer(fmm_plan *plan, int stage, hipStream_t stream) : pl(plan), s(stream)
    {
        if (stage < 0 || !(pl->prof_mask & (1u << stage))) return;
        if ((size_t)(2 * pl->ev_used + 1) >= pl->ev_pool.size()) return;
        pair = pl->ev_used++;
        pl->ev_stage[pair] = stage;
        (void)hipEventRecord(pl->ev_pool[2 * pair], s);
    }
    void stop()
    {
        if (pair >= 0) (void)hipEventRecord(pl->ev_pool[2 * pair + 1], s);
        pair = -1;
    }
    ~StageTimer() { stop(); }
};

// ---- FMM stages (fmm_grid.hip / fmm_points.hip) ----
// Every stage runs for the nr right-hand sides of rh at once (blockIdx.z):
// q, u (and sigma_out) hold nr arrays rh.sv (rh.sr) apart, and the plan's
// workspace must hold nr of them (ensure_rhs).
// q -> u for grid plans: u = -(1/2pi) [ qscale * near(q) + far ], optionally
// also the ring potential.  With defer_l2p the far field is left in the
// leaf-level local expansions (plan->ws.Lt) for grid_ring_source_fmm to add.
int grid_volume_fmm(fmm_plan *plan, const double *q, double qscale, double *u,
                    double *ring_out, bool defer_l2p, const RhsSet &rh, int nr, hipStream_t s);
// second pass: the boundary density from the boundary solve's products
// (plan->shat; also written to plan->ring_q as charges h sigma and to
// sigma_out when given), add its potential to u (and the deferred far field
// of the volume pass when with_volume)
int grid_ring_source_fmm(fmm_plan *plan, double *u, bool with_volume, double *sigma_out,
                         const RhsSet &rh, int nr, hipStream_t s);
// workspace for nr right-hand sides (grows only; drops captured graphs that
// hold the old addresses)
int ensure_rhs(fmm_plan *plan, int nr);
// M2L list split: 1, 2, 4 or 8 blocks per tile (rebuilds the work items,
// grows Lm, drops captured graphs); the default gives half the compute
// units a block
int set_m2l_split(fmm_plan *plan, int split);
int default_m2l_split(const fmm_plan *plan);
// the split a launch over nr right-hand sides takes: the plan's split for
// one, shrunk by nr (rounded down to a power of two) since the right-hand
// sides already multiply the blocks
int m2l_split_for(const fmm_plan *plan, int nr);
// times M2L + the downward launches for every split and keeps the fastest
int tune_m2l_split(fmm_plan *plan, hipStream_t s, int *chosen);
// the right-hand-side set of nr stacked arrays of length sv on this plan
RhsSet plan_rhs(const fmm_plan *plan, int64_t sv, const int *act);
int m2l_kernel_setup(fmm_plan *plan);
int points_fmm(fmm_plan *plan, const double *q, double *u, hipStream_t s);
// Gaussian-bump source model and its parameter gradients (adjoint.hip)
int bumps_eval(fmm_plan *plan, int K, const double *cx, const double *cy, const double *w,
               const double *a, double *f, hipStream_t s);
int bumps_grad(fmm_plan *plan, int K, const double *cx, const double *cy, const double *w,
               const double *a, const double *g, double *gcx, double *gcy, double *gw,
               double *ga, hipStream_t s);
int bumps_grad_noalloc(fmm_plan *plan, int K, const double *cx, const double *cy,
                       const double *w, const double *a, const double *g, double *gcx,
                       double *gcy, double *gw, double *ga, hipStream_t s);
int bumps_scratch_init(fmm_plan *plan);
int points_setup(fmm_plan *plan, const double *dx, const double *dy, hipStream_t s);

// ---- boundary correction (bem.hip) ----
int bem_setup(fmm_plan *plan, hipStream_t s);
int bem_apply(fmm_plan *plan, double *sigma_out, const RhsSet &rh, int nr, hipStream_t s);

// ---- Krylov (krylov.hip) ----
int stencil_apply(fmm_plan *plan, const double *v, double *w, int nr, hipStream_t s);
int gmres_solve(fmm_plan *plan, const double *f, const double *g, double *u,
                const gmres_params *prm, gmres_result *res, hipStream_t s,
                const double *ax = nullptr, const double *ay = nullptr);
int stencil_var_apply(fmm_plan *plan, const double *ax, const double *ay, const double *v,
                      double *w, hipStream_t s);
int gmres_solve_batch(fmm_plan *const *plans, int count, const double *const *f, double *const *u,
                      const gmres_params *prm, gmres_result *res, double *elapsed_ms, bool graphs,
                      bool separate, hipStream_t caller);
int tune_vector_blocks(fmm_plan *plan, hipStream_t s, int *chosen);
void drop_step_graphs(fmm_plan *plan);
int precond_apply_one(fmm_plan *plan, const double *r, double *z, double *phi_ring,
                      double *sigma, hipStream_t s);
// z = P^{-1} r for nr stacked right-hand sides (N apart), those of act only
int precond_apply_rhs(fmm_plan *plan, const double *r, double *z, int nr, int64_t stride,
                      const int *act, hipStream_t s);
// nr stacked solves on one plan (f, u: nr grids of n*n), every launch of a
// step covering all instances (device-side Givens rotations and convergence
// flags); graphs: replay captured steps
int gmres_solve_group(fmm_plan *plan, int nr, const double *const *f, double *const *u,
                      const gmres_params *prm, gmres_result *res, bool graphs, hipStream_t s);
void release_group(fmm_plan *plan);

// Boundary density at node k of side s from the products of the boundary
// solve: sh = [mode 0: even | odd][mode 2: even | odd][mode 1: even | odd]
// (n/2 each).  The mode value at node k is even + odd (k < n/2) or even - odd
// at n-1-k, and sigma_s = (1/4)[ s^_0 + (-1)^s s^_2 + 2 Re(i^s s^_1) ].
__device__ __forceinline__ double ring_sigma(const double2 *__restrict__ sh, int s, int k, int n)
{
    const int m = n >> 1;
    const bool lo = k < m;
    const int kk = lo ? k : n - 1 - k;
    const double sg = lo ? 1.0 : -1.0;
    const double a0 = sh[kk].x + sg * sh[m + kk].x;
    const double a2 = sh[n + kk].x + sg * sh[n + m + kk].x;
    const double2 e1 = sh[2 * n + kk], o1 = sh[2 * n + m + kk];
    const double a1x = e1.x + sg * o1.x, a1y = e1.y + sg * o1.y;
    const double re1 = s == 0 ? a1x : (s == 1 ? -a1y : (s == 2 ? -a1x : a1y));
    return 0.25 * (a0 + ((s & 1) ? -a2 : a2) + 2.0 * re1);
}

// kx(b) + 1 of the plan's near set in 4 bits per b = 0..kMaxK (the form the
// kernels take it in: a runtime shift instead of an indexed array)
inline int near_kx_packed(const fmm_plan *pl)
{
    int v = 0;
    for (int b = 0; b <= kMaxK; ++b) v |= (pl->kx[b] + 1) << (4 * b);
    return v;
}

}  // namespace fmmprec

// p dispatch: instantiates FN<P> for P = 2..20
#define FMM_P_CASE(P, FN, ...) \
    case P:                    \
        return FN<P>(__VA_ARGS__);
#define FMM_DISPATCH_P(p, FN, ...)                                                   \
    switch (p) {                                                                     \
        FMM_P_CASE(2, FN, __VA_ARGS__) FMM_P_CASE(3, FN, __VA_ARGS__)                 \
        FMM_P_CASE(4, FN, __VA_ARGS__) FMM_P_CASE(5, FN, __VA_ARGS__)                 \
        FMM_P_CASE(6, FN, __VA_ARGS__) FMM_P_CASE(7, FN, __VA_ARGS__)                 \
        FMM_P_CASE(8, FN, __VA_ARGS__) FMM_P_CASE(9, FN, __VA_ARGS__)                 \
        FMM_P_CASE(10, FN, __VA_ARGS__) FMM_P_CASE(11, FN, __VA_ARGS__)               \
        FMM_P_CASE(12, FN, __VA_ARGS__) FMM_P_CASE(13, FN, __VA_ARGS__)               \
        FMM_P_CASE(14, FN, __VA_ARGS__) FMM_P_CASE(15, FN, __VA_ARGS__)               \
        FMM_P_CASE(16, FN, __VA_ARGS__) FMM_P_CASE(17, FN, __VA_ARGS__)               \
        FMM_P_CASE(18, FN, __VA_ARGS__) FMM_P_CASE(19, FN, __VA_ARGS__)               \
        FMM_P_CASE(20, FN, __VA_ARGS__)                                              \
        default:                                                                     \
            return FMM_ERR_ARG;                                                      \
    }
