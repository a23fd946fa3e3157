// Krylov solver around the FMM-BEM preconditioner: the 5-point stencil
// (Sec. 2.1, eq. axb) and right-preconditioned FGMRES(m) (GMRES is the
// Krylov method the paper cites in Sec. 1; right preconditioning as in
// Sec. 3.1).
//
// Orthogonalisation is classical Gram-Schmidt applied twice, with the second
// pass and the normalisation of each new vector delayed by one step, so that
// a step makes one reduction and two sweeps over the basis.  Step j holds
// finished vectors v_0..v_{j-1} and a candidate u = V_j that has had one
// projection; it computes z = P u, w = A z and then
//   sweep A: a_i = v_i.u, b_i = v_i.w (i < j), c = u.u, d = u.w, e = w.w
//   (small kernel) rho = sqrt(c - |a|^2), h_j = (d - a.b) / rho,
//                  rt = sqrt(e - |b|^2 - h_j^2)
//   sweep B: v_j = (u - sum a_i v_i) / rho           (second projection of u)
//            u'  = (w - sum b_i v_i - h_j v_j) / rt   (first projection of w)
// w is never stored: both sweeps evaluate the stencil of z on the fly.  The
// host keeps the Hessenberg matrix unrotated; the second projection of u
// corrects the previous column (rows i < j gain rt_prev a_i, the subdiagonal
// becomes rt_prev rho) before the Givens rotations are rebuilt.  The Z
// vectors of the flexible method are P applied to the candidates, which the
// Arnoldi relation A Z = V H accounts for exactly.
//
// Every vector kernel is HBM bound.  Reductions are two-stage with a fixed
// order (no atomics), so repeated solves are bitwise reproducible.  One
// small device-to-host copy per inner iteration feeds the host.
#include <chrono>
#include <cmath>
#include <memory>
#include <thread>
#include <vector>

#include "fmm_internal.h"

namespace fmmprec {

constexpr int kMaxBasis = 32;   // restart <= 32
constexpr int kRedBlocks = 4096;  // partial sums per reduction (coefficient-major)
constexpr int64_t kBasisPad = 256; // elements between consecutive basis vectors beyond n^2
constexpr int kPartRows = 2 * kMaxBasis + 4;

// layout of plan->dscal (device) / plan->hpin (host mirror)
constexpr int kRaw = 0;     // a_0..a_{j-1}, b_0..b_{j-1}, c, d, e
constexpr int kOut = 72;    // rho, h_j, rt
constexpr int kCoef = 80;   // sweep-B coefficients: 1/rho, 1/rt, -h_j/(rho rt), -a_i/rho, -(b_i - h_j a_i/rho)/rt
constexpr int kScal = 160;  // norms
// pinned host mirror: two slots of kHostSlot doubles; step j's scalars land in
// slot j & 1, so that step j + 1 may run (and copy) while the host reads j's
constexpr int kHostSlot = 256;
// a step is issued ahead of the host's decision when the residual estimate is
// above this multiple of the tolerance (one more step cannot reach it) or,
// once a step of the cycle has shown the rate, above kSpecSafety times the
// largest of the last two per-step reductions (one more step at that rate
// stays a factor kSpecSafety above the tolerance)
constexpr double kSpecMargin = 1e3;
constexpr double kSpecSafety = 4.0;

// Instances of a group solve (many right-hand sides on one plan), selected by
// blockIdx.y of the vector kernels and by blockIdx.x of the per-instance
// scalar kernels: basis vectors V vs doubles apart, Z vectors zs, grid
// vectors (b, x, w) xs, reduction partials ps, scalar slots ds.  act (device,
// may be null) flags the instances that take part in a launch; the blocks of
// the others return at once.  A lone solve passes the defaults.
struct Inst {
    int64_t vs = 0, zs = 0, xs = 0, ps = 0, ds = 0;
    const int *act = nullptr;
};
__device__ __forceinline__ bool inst_on(const Inst &in, int r) { return !in.act || in.act[r] != 0; }

__global__ __launch_bounds__(256) void k_stencil(const double *__restrict__ v,
                                                 double *__restrict__ w, int n, double ih2)
{
    v += (size_t)blockIdx.z * n * n;
    w += (size_t)blockIdx.z * n * n;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const size_t e = (size_t)j * n + i;
    double c = 4.0 * v[e];
    if (i > 0) c -= v[e - 1];
    if (i < n - 1) c -= v[e + 1];
    if (j > 0) c -= v[e - n];
    if (j < n - 1) c -= v[e + n];
    w[e] = c * ih2;
}

// Face coefficients of the variable-coefficient operator (null: constant
// coefficient 1): ax[j (n+1) + i] sits between nodes i-1 and i of row j,
// ay[j n + i] between rows j-1 and j of column i.
struct Faces {
    const double *ax, *ay;
};

// h^2 (A v)_e at element e of a row-major n x n grid, n = 2^ln; VAR selects
// the flux form sum_faces a_f (v_e - v_neighbour) (Sec. 6.4), otherwise the
// plain 5-point stencil (Sec. 2.1); values outside the grid are zero.
template <bool VAR>
__device__ __forceinline__ double stencil_at(const double *__restrict__ v, uint32_t e, int n, int ln,
                                             Faces fc)
{
    const uint32_t i = e & (uint32_t)(n - 1), j = e >> ln;
    const double ve = v[e];
    const double vw = i > 0 ? v[e - 1] : 0.0, vE = i < (uint32_t)n - 1 ? v[e + 1] : 0.0;
    const double vs = j > 0 ? v[e - n] : 0.0, vn = j < (uint32_t)n - 1 ? v[e + n] : 0.0;
    if (!VAR) return 4.0 * ve - vw - vE - vs - vn;
    const double *axr = fc.ax + (size_t)j * (n + 1) + i;
    const double *ayc = fc.ay + (size_t)j * n + i;
    return axr[1] * (ve - vE) + axr[0] * (ve - vw) + ayc[n] * (ve - vn) + ayc[0] * (ve - vs);
}

// block-level sum of NV per-thread values into part[i * kRedBlocks + blockIdx.x]
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double *part)
{
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double a = acc[i];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if (lane == 0) red[wv][i] = a;
    }
    __syncthreads();
    if (threadIdx.x < NV)
        part[(size_t)threadIdx.x * kRedBlocks + blockIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// sweep A of step NJ: partial sums of a_i, b_i (i < NJ), c, d, e with
// u = V_NJ and w = A z (scaled by 1/h^2)
template <int NJ, bool VAR>
__global__ __launch_bounds__(256) void k_arnoldi_dots(const double *__restrict__ z,
                                                      const double *__restrict__ V, int64_t ldv,
                                                      double *__restrict__ part, int n, int ln,
                                                      double ih2, Faces fc, Inst in)
{
    if (!inst_on(in, blockIdx.y)) return;
    z += blockIdx.y * in.zs;
    V += blockIdx.y * in.vs;
    part += blockIdx.y * in.ps;
    constexpr int NA = 2 * NJ + 3;
    const uint32_t N = (uint32_t)n << ln;
    double acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.0;
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < N; e += gridDim.x * 256u) {
        double vv[NJ > 0 ? NJ : 1];
#pragma unroll
        for (int i = 0; i < NJ; ++i) vv[i] = V[i * ldv + e];
        const double u = V[NJ * ldv + e];
        const double w = stencil_at<VAR>(z, e, n, ln, fc) * ih2;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            acc[i] = fma(vv[i], u, acc[i]);
            acc[NJ + i] = fma(vv[i], w, acc[NJ + i]);
        }
        acc[2 * NJ] = fma(u, u, acc[2 * NJ]);
        acc[2 * NJ + 1] = fma(u, w, acc[2 * NJ + 1]);
        acc[2 * NJ + 2] = fma(w, w, acc[2 * NJ + 2]);
    }
    block_reduce_store<NA>(acc, part);
}

// The block partials of sweep A reduced to a_i, b_i, c, d, e (one wave per
// row, lanes in a fixed order, then a shuffle tree), and from them rho, h_j,
// rt and the sweep-B coefficients: one launch between the two sweeps.
__global__ __launch_bounds__(1024) void k_arnoldi_coef(const double *__restrict__ part, int nblk,
                                                       double *__restrict__ d, int nj, Inst in)
{
    if (!inst_on(in, blockIdx.x)) return;
    part += blockIdx.x * in.ps;
    d += blockIdx.x * in.ds;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wv; i < 2 * nj + 3; i += 16) {
        const double *pi = part + (size_t)i * kRedBlocks;
        double acc = 0.0;
#pragma unroll 8
        for (int b = lane; b < nblk; b += 64) acc += pi[b];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) d[kRaw + i] = acc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double *a = d + kRaw, *b = d + kRaw + nj;
    const double c = d[kRaw + 2 * nj], ud = d[kRaw + 2 * nj + 1], e = d[kRaw + 2 * nj + 2];
    double sa = 0.0, sb = 0.0, sab = 0.0;
    for (int i = 0; i < nj; ++i) {
        sa = fma(a[i], a[i], sa);
        sb = fma(b[i], b[i], sb);
        sab = fma(a[i], b[i], sab);
    }
    const double rho2 = c - sa;
    const double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
    const double irho = rho > 0.0 ? 1.0 / rho : 0.0;
    const double hj = (ud - sab) * irho;
    const double rt2 = e - sb - hj * hj;
    const double rt = rt2 > 0.0 ? sqrt(rt2) : 0.0;
    const double irt = rt > 0.0 ? 1.0 / rt : 0.0;
    d[kOut] = rho;
    d[kOut + 1] = hj;
    d[kOut + 2] = rt;
    double *cf = d + kCoef;
    cf[0] = irho;
    cf[1] = irt;
    cf[2] = -hj * irho * irt;
    for (int i = 0; i < nj; ++i) {
        cf[3 + i] = -a[i] * irho;
        cf[3 + nj + i] = -(b[i] - hj * a[i] * irho) * irt;
    }
}

// sweep B of step NJ: V_NJ <- v_NJ (finished), V_NJ+1 <- next candidate
template <int NJ, bool VAR>
__global__ __launch_bounds__(256) void k_arnoldi_update(const double *__restrict__ z,
                                                        double *__restrict__ V, int64_t ldv,
                                                        const double *__restrict__ cf, int n,
                                                        int ln, double ih2, Faces fc, Inst in)
{
    if (!inst_on(in, blockIdx.y)) return;
    z += blockIdx.y * in.zs;
    V += blockIdx.y * in.vs;
    cf += blockIdx.y * in.ds;
    const uint32_t N = (uint32_t)n << ln;
    const double cu = cf[0], cw = cf[1], cuu = cf[2];
    double cv[NJ > 0 ? NJ : 1], cn[NJ > 0 ? NJ : 1];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        cv[i] = cf[3 + i];
        cn[i] = cf[3 + NJ + i];
    }
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < N; e += gridDim.x * 256u) {
        double vv[NJ > 0 ? NJ : 1];
#pragma unroll
        for (int i = 0; i < NJ; ++i) vv[i] = V[i * ldv + e];
        const double u = V[NJ * ldv + e];
        const double w = stencil_at<VAR>(z, e, n, ln, fc) * ih2;
        double vj = cu * u, un = fma(cuu, u, cw * w);
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            vj = fma(cv[i], vv[i], vj);
            un = fma(cn[i], vv[i], un);
        }
        V[NJ * ldv + e] = vj;
        V[(NJ + 1) * ldv + e] = un;
    }
}

#define KRY_NJ_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) \
    X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31)

template <bool VAR>
static void launch_arnoldi_dots(int nj, dim3 g, hipStream_t s, const double *z, const double *V,
                                int64_t ldv, double *part, int n, int ln, double ih2, Faces fc,
                                const Inst &in = Inst{})
{
    switch (nj) {
#define X(k) case k: hipLaunchKernelGGL((k_arnoldi_dots<k, VAR>), g, dim3(256), 0, s, z, V, ldv, part, n, ln, ih2, fc, in); break;
        KRY_NJ_CASES(X)
#undef X
    }
}

template <bool VAR>
static void launch_arnoldi_update(int nj, dim3 g, hipStream_t s, const double *z, double *V,
                                  int64_t ldv, const double *cf, int n, int ln, double ih2, Faces fc,
                                  const Inst &in = Inst{})
{
    switch (nj) {
#define X(k) case k: hipLaunchKernelGGL((k_arnoldi_update<k, VAR>), g, dim3(256), 0, s, z, V, ldv, cf, n, ln, ih2, fc, in); break;
        KRY_NJ_CASES(X)
#undef X
    }
}

// r = b - A x, partial r.r
template <bool VAR>
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ b,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ r,
                                                  double *__restrict__ part, int n, int ln,
                                                  double ih2, Faces fc, Inst in)
{
    if (!inst_on(in, blockIdx.y)) return;
    b += blockIdx.y * in.xs;
    x += blockIdx.y * in.xs;
    r += blockIdx.y * in.xs;
    part += blockIdx.y * in.ps;
    const uint32_t N = (uint32_t)n << ln;
    double acc[1] = {0.0};
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < N; e += gridDim.x * 256u) {
        const double re = b[e] - stencil_at<VAR>(x, e, n, ln, fc) * ih2;
        r[e] = re;
        acc[0] = fma(re, re, acc[0]);
    }
    block_reduce_store<1>(acc, part);
}

// w = A v with face coefficients
__global__ __launch_bounds__(256) void k_stencil_var(const double *__restrict__ v,
                                                     double *__restrict__ w, int n, int ln,
                                                     double ih2, Faces fc)
{
    const uint32_t N = (uint32_t)n << ln;
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < N; e += gridDim.x * 256u)
        w[e] = stencil_at<true>(v, e, n, ln, fc) * ih2;
}

// partial v.v
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ v,
                                               double *__restrict__ part, int64_t N, Inst in)
{
    if (!inst_on(in, blockIdx.y)) return;
    v += blockIdx.y * in.xs;
    part += blockIdx.y * in.ps;
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256)
        acc[0] = fma(v[e], v[e], acc[0]);
    block_reduce_store<1>(acc, part);
}

// out[i] = sqrt(sum_b part[i][b]) (a norm from its block partials).  One
// block per row i; the summation order is fixed.
__global__ __launch_bounds__(256) void k_finish(const double *__restrict__ part, int nblk,
                                                double *__restrict__ out)
{
    __shared__ double red[4];
    const int i = blockIdx.x;
    const double *pi = part + (size_t)i * kRedBlocks;
    double a = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nblk; b += 256) a += pi[b];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) out[i] = sqrt((red[0] + red[1]) + (red[2] + red[3]));
}

// y = x * (1 / *scal) or y = x * c
__global__ void k_scale(const double *__restrict__ x, double *__restrict__ y,
                        const double *__restrict__ scal, double c, int64_t N)
{
    const double f = scal ? 1.0 / scal[0] : c;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256)
        y[e] = x[e] * f;
}

struct Coef {
    double c[kMaxBasis];
};

// x += sum_i y_i Z_i
__global__ __launch_bounds__(256) void k_axpy_multi(const double *__restrict__ Z, int64_t ldz,
                                                    int k, Coef y, double *__restrict__ x,
                                                    int64_t N)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        double a = x[e];
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i)
            if (i < k) a = fma(y.c[i], Z[i * ldz + e], a);
        x[e] = a;
    }
}

// b = f + (Dirichlet values at the neighbouring ring nodes) / h^2
__global__ void k_make_rhs(const double *__restrict__ f, const double *__restrict__ g,
                           double *__restrict__ b, int n, double ih2)
{
    const int64_t N = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        double v = f[e];
        if (g) {
            const int i = (int)(e % n), j = (int)(e / n);
            double add = 0.0;
            if (j == 0) add += g[i];                    // bottom node k = i
            if (i == n - 1) add += g[n + j];            // right node k = j
            if (j == n - 1) add += g[2 * n + (n - 1 - i)];  // top node at x = (i+1)h: k = n-1-i
            if (i == 0) add += g[3 * n + (n - 1 - j)];  // left node at y = (j+1)h: k = n-1-j
            v += add * ih2;
        }
        b[e] = v;
    }
}

// blocks of the vector kernels: the plan's tuned count, else one per 1024 elements
static int red_blocks(const fmm_plan *pl, int64_t N)
{
    if (pl && pl->vec_blocks > 0) return pl->vec_blocks;
    int64_t b = (N + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    return (int)b;
}

int stencil_var_apply(fmm_plan *pl, const double *ax, const double *ay, const double *v, double *w,
                      hipStream_t s)
{
    const int n = (int)pl->n;
    const double ih2 = 1.0 / (pl->h * pl->h);
    StageTimer t(pl, FMM_STAGE_STENCIL, s);
    hipLaunchKernelGGL(k_stencil_var, dim3(red_blocks(pl, (int64_t)n * n)), dim3(256), 0, s, v, w, n,
                       pl->L + 3, ih2, Faces{ax, ay});
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int stencil_apply(fmm_plan *pl, const double *v, double *w, int nr, hipStream_t s)
{
    const int n = (int)pl->n;
    const double ih2 = 1.0 / (pl->h * pl->h);
    StageTimer t(pl, FMM_STAGE_STENCIL, s);
    hipLaunchKernelGGL(k_stencil, dim3((n + 63) / 64, (n + 3) / 4, nr), dim3(256), 0, s, v, w, n, ih2);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int precond_apply_one(fmm_plan *pl, const double *r, double *z, double *phi_ring, double *sigma,
                      hipStream_t s)
{
    const double h2 = pl->h * pl->h;
    const bool need_ring = pl->bem || phi_ring;
    const RhsSet rh = plan_rhs(pl, pl->n * pl->n, nullptr);
    int st = grid_volume_fmm(pl, r, h2, z, need_ring ? pl->phi_ring : nullptr, pl->bem != 0, rh, 1, s);
    if (st != FMM_OK) return st;
    if (phi_ring)
        FMM_HIP(pl, hipMemcpyAsync(phi_ring, pl->phi_ring, 4 * (size_t)pl->n * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
    if (pl->bem) {
        st = bem_apply(pl, sigma, rh, 1, s);
        if (st != FMM_OK) return st;
        st = grid_ring_source_fmm(pl, z, true, sigma, rh, 1, s);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

int precond_apply_rhs(fmm_plan *pl, const double *r, double *z, int nr, int64_t stride,
                      const int *act, hipStream_t s)
{
    int st = ensure_rhs(pl, nr);
    if (st != FMM_OK) return st;
    const double h2 = pl->h * pl->h;
    const RhsSet rh = plan_rhs(pl, stride, act);
    st = grid_volume_fmm(pl, r, h2, z, pl->bem ? pl->phi_ring : nullptr, pl->bem != 0, rh, nr, s);
    if (st != FMM_OK) return st;
    if (pl->bem) {
        st = bem_apply(pl, nullptr, rh, nr, s);
        if (st != FMM_OK) return st;
        st = grid_ring_source_fmm(pl, z, true, nullptr, rh, nr, s);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

void drop_step_graphs(fmm_plan *pl)
{
    for (auto &ex : pl->step_exec)
        if (ex) (void)hipGraphExecDestroy(ex);
    pl->step_exec.clear();
    for (auto &ex : pl->g_step_exec)
        if (ex) (void)hipGraphExecDestroy(ex);
    pl->g_step_exec.clear();
    if (pl->g_end_exec) (void)hipGraphExecDestroy(pl->g_end_exec);
    pl->g_end_exec = nullptr;
    pl->g_graph_nr = 0;
}

static int ensure_krylov(fmm_plan *pl, int m)
{
    if (pl->kry_m >= m) return FMM_OK;
    drop_step_graphs(pl);   // the captured steps hold the old basis addresses
    const size_t N = (size_t)pl->n * pl->n;
    if (pl->V) { hipFree(pl->V); pl->V = nullptr; }
    if (pl->Z) { hipFree(pl->Z); pl->Z = nullptr; }
    if (!pl->w) FMM_HIP(pl, hipMalloc(&pl->w, N * sizeof(double)));
    if (!pl->b) FMM_HIP(pl, hipMalloc(&pl->b, N * sizeof(double)));
    if (!pl->partial) FMM_HIP(pl, hipMalloc(&pl->partial, (size_t)kRedBlocks * kPartRows * sizeof(double)));
    if (!pl->dscal) FMM_HIP(pl, hipMalloc(&pl->dscal, 256 * sizeof(double)));
    if (!pl->hpin)
        FMM_HIP(pl, hipHostMalloc((void **)&pl->hpin, 2 * kHostSlot * sizeof(double), hipHostMallocDefault));
    for (int i = 0; i < 2; ++i)
        if (!pl->sevent[i]) FMM_HIP(pl, hipEventCreateWithFlags(&pl->sevent[i], hipEventDisableTiming));
    // vectors n^2 = 2^(2k) elements apart would start on the same memory
    // channels, and the sweeps stream up to m + 2 of them side by side
    pl->ldb = (int64_t)N + kBasisPad;
    hipError_t e1 = hipMalloc(&pl->V, (size_t)(m + 1) * pl->ldb * sizeof(double));
    if (e1 != hipSuccess) return fail(pl, FMM_ERR_ALLOC, "Krylov basis allocation failed");
    hipError_t e2 = hipMalloc(&pl->Z, (size_t)m * pl->ldb * sizeof(double));
    if (e2 != hipSuccess) return fail(pl, FMM_ERR_ALLOC, "Krylov basis allocation failed");
    pl->kry_m = m;
    return FMM_OK;
}


// Resumable FGMRES(m) on one plan.  Each issue_*() enqueues a chunk of GPU
// work on the solve's stream that ends with a device-to-host copy into the
// plan's pinned buffer; advance() is called once that work has completed,
// consumes the copied scalars on the host and enqueues the next chunk:
//   INIT  b and |b|
//   RES   true residual r = b - A u and |r| (start of a cycle)
//   STEP  one Arnoldi step j (preconditioner, both sweeps, coefficients)
// A single solve drives it with a stream synchronisation per chunk; the
// batch loop interleaves many solves on their own streams.  With graphs,
// step j of a plan is captured once into a HIP graph and replayed.
//
// With spec (single solves), step j + 1 is issued before the host has read
// step j's scalars whenever step j - 1 left the residual estimate far above
// the tolerance; the host then waits for step j's event only, and the GPU
// runs on while it does the Givens update.  A step issued this way that turns
// out not to be needed only writes basis vectors beyond the cycle's last one.
class Fgmres {
  public:
    Fgmres(fmm_plan *pl, const double *f, const double *g, double *u, const gmres_params &prm,
           hipStream_t s, Faces fc, bool graphs, bool spec = false)
        : pl_(pl), f_(f), g_(g), u_(u), tol_(prm.tol), m_(prm.restart), maxit_(prm.maxit), s_(s),
          fc_(fc), var_(fc.ax != nullptr), graphs_(graphs), spec_(spec && !graphs)
    {
    }

    // waits for the work advance() consumes next
    int wait()
    {
        if (phase_ == STEP && spec_) {
            FMM_HIP(pl_, hipEventSynchronize(pl_->sevent[j_ & 1]));
        } else {
            FMM_HIP(pl_, hipStreamSynchronize(s_));
        }
        return FMM_OK;
    }

    int begin()
    {
        int st = ensure_krylov(pl_, m_);
        if (st != FMM_OK) return st;
        n_ = (int)pl_->n;
        N_ = (int64_t)n_ * n_;
        ih2_ = 1.0 / (pl_->h * pl_->h);
        ln_ = pl_->L + 3;
        nblk_ = red_blocks(pl_, N_);
        Hr_.assign((size_t)(m_ + 1) * m_, 0.0);
        H_ = Hr_;
        cs_.assign(m_, 0.0);
        sn_.assign(m_, 0.0);
        gg_.assign(m_ + 1, 0.0);
        y_.assign(m_, 0.0);
        hipLaunchKernelGGL(k_make_rhs, dim3(nblk_), dim3(256), 0, s_, f_, g_, pl_->b, n_, ih2_);
        hipLaunchKernelGGL(k_sumsq, dim3(nblk_), dim3(256), 0, s_, pl_->b, pl_->partial, N_, Inst{});
        phase_ = INIT;
        return fetch_scalar();
    }

    int advance()
    {
        FMM_HIP(pl_, hipGetLastError());
        switch (phase_) {
        case INIT:
            bnorm_ = pl_->hpin[kScal];
            if (!std::isfinite(bnorm_)) return fail(pl_, FMM_ERR_NUMERIC, "right-hand side is not finite");
            if (bnorm_ == 0.0) {
                FMM_HIP(pl_, hipMemsetAsync(u_, 0, N_ * sizeof(double), s_));
                status_ = FMM_OK;
                phase_ = DONE;
                return FMM_OK;
            }
            return issue_residual();
        case RES: {
            const double beta = pl_->hpin[kScal];
            if (!std::isfinite(beta)) return fail(pl_, FMM_ERR_NUMERIC, "residual is not finite");
            r_.true_rel_res = beta / bnorm_;
            if (beta / bnorm_ <= tol_ || iters_ >= maxit_) {
                status_ = beta / bnorm_ <= tol_ ? FMM_OK : FMM_NOT_CONVERGED;
                phase_ = DONE;
                return FMM_OK;
            }
            hipLaunchKernelGGL(k_scale, dim3(nblk_), dim3(256), 0, s_, pl_->w, pl_->V, nullptr,
                               1.0 / beta, N_);
            std::fill(Hr_.begin(), Hr_.end(), 0.0);
            beta_ = beta;
            rt_prev_ = 0.0;
            j_ = 0;
            ahead_ = -1;
            const int st = issue_step();
            if (st != FMM_OK) return st;
            return issue_ahead(beta / bnorm_);
        }
        case STEP: {
            int st = consume_step();
            if (st != FMM_OK) return st;
            if (est_ <= tol_ || rt_last_ == 0.0 || j_ + 1 == m_ || iters_ >= maxit_) {
                finish_cycle();
                return issue_residual();
            }
            ++j_;
            if (ahead_ != j_) {
                st = issue_step();
                if (st != FMM_OK) return st;
            }
            return issue_ahead(est_);
        }
        case DONE:
            break;
        }
        return FMM_OK;
    }

    bool done() const { return phase_ == DONE; }
    int status() const { return status_; }
    gmres_result result() const
    {
        gmres_result r = r_;
        r.iters = iters_;
        r.est_rel_res = est_;
        return r;
    }

  private:
    enum Phase { INIT, RES, STEP, DONE };

    int fetch_scalar()
    {
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s_, pl_->partial, nblk_, pl_->dscal + kScal);
        FMM_HIP(pl_, hipMemcpyAsync(pl_->hpin + kScal, pl_->dscal + kScal, sizeof(double),
                                    hipMemcpyDeviceToHost, s_));
        return FMM_OK;
    }

    int issue_residual()
    {
        {
            StageTimer t(pl_, FMM_STAGE_STENCIL, s_);
            if (var_)
                hipLaunchKernelGGL(k_residual<true>, dim3(nblk_), dim3(256), 0, s_, pl_->b, u_, pl_->w,
                                   pl_->partial, n_, ln_, ih2_, fc_, Inst{});
            else
                hipLaunchKernelGGL(k_residual<false>, dim3(nblk_), dim3(256), 0, s_, pl_->b, u_, pl_->w,
                                   pl_->partial, n_, ln_, ih2_, fc_, Inst{});
        }
        phase_ = RES;
        return fetch_scalar();
    }

    // the launches of Arnoldi step j (identical on every call, so capturable)
    // with spec: step j_ + 1 now, if an estimate of est leaves it certainly needed
    int issue_ahead(double est)
    {
        const double rmax = std::max(red_[0], red_[1]);
        const double margin = rmax > 1.0 ? std::min(kSpecMargin, kSpecSafety * rmax) : kSpecMargin;
        if (!spec_ || j_ + 1 >= m_ || iters_ + 2 > maxit_ || !(est > tol_ * margin)) return FMM_OK;
        ahead_ = j_ + 1;
        return launch_step(j_ + 1);
    }

    int launch_step(int j)
    {
        const int64_t ld = pl_->ldb;
        double *uj = pl_->V + (size_t)j * ld, *zj = pl_->Z + (size_t)j * ld;
        int st = precond_apply_one(pl_, uj, zj, nullptr, nullptr, s_);
        if (st != FMM_OK) return st;
        StageTimer ta(pl_, FMM_STAGE_ARNOLDI, s_);
        const dim3 gv(nblk_);
        if (var_)
            launch_arnoldi_dots<true>(j, gv, s_, zj, pl_->V, ld, pl_->partial, n_, ln_, ih2_, fc_);
        else
            launch_arnoldi_dots<false>(j, gv, s_, zj, pl_->V, ld, pl_->partial, n_, ln_, ih2_, fc_);
        hipLaunchKernelGGL(k_arnoldi_coef, dim3(1), dim3(1024), 0, s_, pl_->partial, nblk_,
                           pl_->dscal, j, Inst{});
        if (var_)
            launch_arnoldi_update<true>(j, gv, s_, zj, pl_->V, ld, pl_->dscal + kCoef, n_, ln_, ih2_, fc_);
        else
            launch_arnoldi_update<false>(j, gv, s_, zj, pl_->V, ld, pl_->dscal + kCoef, n_, ln_, ih2_, fc_);
        ta.stop();
        FMM_HIP(pl_, hipMemcpyAsync(pl_->hpin + kHostSlot * (j & 1), pl_->dscal,
                                    kCoef * sizeof(double), hipMemcpyDeviceToHost, s_));
        if (spec_) FMM_HIP(pl_, hipEventRecord(pl_->sevent[j & 1], s_));
        return FMM_OK;
    }

    int issue_step()
    {
        phase_ = STEP;
        if (!graphs_) return launch_step(j_);
        if ((int)pl_->step_exec.size() < m_) pl_->step_exec.resize(m_, nullptr);
        hipGraphExec_t &ex = pl_->step_exec[j_];
        if (!ex) {
            hipGraph_t gr = nullptr;
            FMM_HIP(pl_, hipStreamBeginCapture(s_, hipStreamCaptureModeRelaxed));
            const int st = launch_step(j_);
            const hipError_t ec = hipStreamEndCapture(s_, &gr);
            if (st != FMM_OK) {
                if (gr) (void)hipGraphDestroy(gr);
                return st;
            }
            FMM_HIP(pl_, ec);
            const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            FMM_HIP(pl_, ei);
        }
        FMM_HIP(pl_, hipGraphLaunch(ex, s_));
        return FMM_OK;
    }

    int consume_step()
    {
        const int j = j_, m = m_;
        const double *hs = pl_->hpin + kHostSlot * (j & 1);
        const double *a = hs + kRaw, *bb = hs + kRaw + j;
        const double rho = hs[kOut], hj = hs[kOut + 1], rt = hs[kOut + 2];
        if (!(rho > 0.0) || !std::isfinite(rho) || !std::isfinite(hj) || !std::isfinite(rt))
            return fail(pl_, FMM_ERR_NUMERIC, "Arnoldi produced a non-finite or zero norm");
        if (j == 0) {
            g0_ = beta_ * rho;             // r = beta u_0 = beta rho v_0
        } else {                           // second projection of u_j fixes column j - 1
            for (int i = 0; i < j; ++i) Hr_[(size_t)i * m + j - 1] += rt_prev_ * a[i];
            Hr_[(size_t)j * m + j - 1] = rt_prev_ * rho;
        }
        for (int i = 0; i < j; ++i) Hr_[(size_t)i * m + j] = bb[i];
        Hr_[(size_t)j * m + j] = hj;
        Hr_[(size_t)(j + 1) * m + j] = rt;
        rt_prev_ = rt;
        rt_last_ = rt;
        // Givens QR of columns 0..j
        H_ = Hr_;
        std::fill(gg_.begin(), gg_.end(), 0.0);
        gg_[0] = g0_;
        for (int c = 0; c <= j; ++c) {
            for (int i = 0; i < c; ++i) {
                const double x0 = H_[(size_t)i * m + c], x1 = H_[(size_t)(i + 1) * m + c];
                H_[(size_t)i * m + c] = cs_[i] * x0 + sn_[i] * x1;
                H_[(size_t)(i + 1) * m + c] = -sn_[i] * x0 + cs_[i] * x1;
            }
            const double x0 = H_[(size_t)c * m + c], x1 = H_[(size_t)(c + 1) * m + c];
            const double rr = std::hypot(x0, x1);
            cs_[c] = x0 / rr;
            sn_[c] = x1 / rr;
            H_[(size_t)c * m + c] = rr;
            H_[(size_t)(c + 1) * m + c] = 0.0;
            gg_[c + 1] = -sn_[c] * gg_[c];
            gg_[c] = cs_[c] * gg_[c];
        }
        ++iters_;
        const double prev = j == 0 ? beta_ / bnorm_ : est_;
        est_ = std::fabs(gg_[j + 1]) / bnorm_;
        // the step's reduction of the estimate (the cycle's first step counts
        // from the residual it restarted from)
        red_[j & 1] = est_ > 0.0 ? prev / est_ : 0.0;
        if (j == 0) red_[1] = 0.0;
        return FMM_OK;
    }

    // least squares of the cycle and u += Z y
    void finish_cycle()
    {
        const int k = j_ + 1, m = m_;
        for (int i = k - 1; i >= 0; --i) {
            double sacc = gg_[i];
            for (int t = i + 1; t < k; ++t) sacc -= H_[(size_t)i * m + t] * y_[t];
            y_[i] = sacc / H_[(size_t)i * m + i];
        }
        Coef cy{};
        for (int i = 0; i < k; ++i) cy.c[i] = y_[i];
        hipLaunchKernelGGL(k_axpy_multi, dim3(nblk_), dim3(256), 0, s_, pl_->Z, pl_->ldb, k, cy, u_, N_);
        r_.restarts++;
    }

    fmm_plan *pl_;
    const double *f_, *g_;
    double *u_;
    double tol_;
    int m_, maxit_;
    hipStream_t s_;
    Faces fc_;
    bool var_, graphs_, spec_;
    int ahead_ = -1;   // step issued ahead of the host's decision, or -1
    int n_ = 0, ln_ = 0, nblk_ = 1;
    int64_t N_ = 0;
    double ih2_ = 0.0;
    std::vector<double> Hr_, H_, cs_, sn_, gg_, y_;
    Phase phase_ = INIT;
    int iters_ = 0, j_ = 0, status_ = FMM_NOT_CONVERGED;
    double bnorm_ = 0.0, beta_ = 0.0, g0_ = 0.0, rt_prev_ = 0.0, rt_last_ = 0.0, est_ = 1.0;
    double red_[2] = {0.0, 0.0};   // reductions of the estimate by the last two steps
    gmres_result r_{};
};

int gmres_solve(fmm_plan *pl, const double *f, const double *g, double *u, const gmres_params *prm,
                gmres_result *res, hipStream_t s, const double *ax, const double *ay)
{
    Fgmres sol(pl, f, g, u, *prm, s, Faces{ax, ay}, false, true);
    int st = sol.begin();
    while (st == FMM_OK && !sol.done()) {
        st = sol.wait();
        if (st == FMM_OK) st = sol.advance();
    }
    if (st != FMM_OK) return st;
    FMM_HIP(pl, hipStreamSynchronize(s));
    if (res) *res = sol.result();
    return sol.status();
}

static int gmres_solve_batch_separate(fmm_plan *const *plans, int count, const double *const *f,
                                      double *const *u, const gmres_params *prm, gmres_result *res,
                                      double *elapsed_ms, bool graphs, hipStream_t caller)
{
    std::vector<std::unique_ptr<Fgmres>> sv(count);
    std::vector<char> fin(count, 0);
    hipEvent_t start = nullptr;
    fmm_plan *p0 = plans[0];
    FMM_HIP(p0, hipEventCreateWithFlags(&start, hipEventDisableTiming));
    FMM_HIP(p0, hipEventRecord(start, caller));
    int st = FMM_OK;
    for (int i = 0; i < count && st == FMM_OK; ++i) {
        fmm_plan *pl = plans[i];
        if (!pl->bstream && hipStreamCreateWithFlags(&pl->bstream, hipStreamNonBlocking) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "stream creation failed");
        if (st == FMM_OK && !pl->bevent &&
            hipEventCreateWithFlags(&pl->bevent, hipEventDisableTiming) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "event creation failed");
        if (st == FMM_OK && hipStreamWaitEvent(pl->bstream, start, 0) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "stream wait failed");
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < count && st == FMM_OK; ++i) {
        fmm_plan *pl = plans[i];
        sv[i].reset(new Fgmres(pl, f[i], nullptr, u[i], *prm, pl->bstream, Faces{nullptr, nullptr},
                               graphs && pl->prof_mask == 0));
        st = sv[i]->begin();
        if (st == FMM_OK && hipEventRecord(pl->bevent, pl->bstream) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "event record failed");
    }
    int active = count, failed_at = -1;
    while (st == FMM_OK && active > 0) {
        bool moved = false;
        for (int i = 0; i < count && st == FMM_OK; ++i) {
            if (fin[i]) continue;
            fmm_plan *pl = plans[i];
            const hipError_t q = hipEventQuery(pl->bevent);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                st = fail(pl, FMM_ERR_DEVICE, hipGetErrorString(q));
                failed_at = i;
                break;
            }
            moved = true;
            st = sv[i]->advance();
            if (st != FMM_OK) {
                failed_at = i;
                break;
            }
            if (hipEventRecord(pl->bevent, pl->bstream) != hipSuccess) {
                st = fail(pl, FMM_ERR_DEVICE, "event record failed");
                failed_at = i;
                break;
            }
            if (sv[i]->done()) {
                fin[i] = 1;
                --active;
                if (elapsed_ms)
                    elapsed_ms[i] = std::chrono::duration<double, std::milli>(
                                        std::chrono::steady_clock::now() - t0).count();
                if (res) res[i] = sv[i]->result();
            }
        }
        if (!moved) std::this_thread::yield();
    }
    // every instance stream drains before the caller's stream goes on
    int overall = FMM_OK;
    for (int i = 0; i < count; ++i) {
        fmm_plan *pl = plans[i];
        if (!pl->bstream) continue;
        if (pl->bevent) {
            (void)hipEventRecord(pl->bevent, pl->bstream);
            (void)hipStreamWaitEvent(caller, pl->bevent, 0);
        }
        if (st != FMM_OK) (void)hipStreamSynchronize(pl->bstream);
        if (st == FMM_OK && sv[i] && sv[i]->status() != FMM_OK) overall = FMM_NOT_CONVERGED;
    }
    (void)hipEventDestroy(start);
    if (st != FMM_OK) {
        if (failed_at > 0) p0->err = plans[failed_at]->err;
        return st;
    }
    return overall;
}


// ---------------------------------------------------------------------------
// Group solves: nr right-hand sides of one plan solved together.  Every
// launch of an Arnoldi step covers all instances (blockIdx.y of the vector
// kernels, blockIdx.z of the FMM kernels, blockIdx.x of the scalar kernels),
// and the host's part of a step, the Givens rotations and the convergence
// test, runs on the device, one wave per instance.  An instance whose cycle
// has ended clears its run flag; the blocks of every later launch return at
// once for it, so a captured step replays unchanged for any subset of the
// instances.  The host reads the run flags once per step (a copy into pinned
// memory at the end of the captured step) to decide whether another step is
// needed, and once per cycle the statuses.
//
// Per instance, the device keeps the rotated Hessenberg columns R, the
// unrotated last column (the delayed second projection corrects it one step
// later, see the Arnoldi kernels above), the rotations, the rotated
// right-hand side g and the scalars of the cycle.  Step j:
//   1. column j-1 gets its correction (rows i < j gain rt_prev a_i, row j
//      becomes rt_prev rho), the committed rotations 0..j-2, and its own
//      rotation, which is committed (g[j-1], g[j] updated);
//   2. column j (b_i, h_j, rt) is rotated by 0..j-1 and a tentative rotation
//      gives the residual estimate |sn g[j]| / |b|;
//   3. the cycle ends when the estimate reaches the tolerance, rt = 0, the
//      basis is full or maxit is spent: the least-squares solution uses the
//      committed columns and the tentative last one.
// At the end of a cycle: y = R^-1 g, x += Z y, the true residual, and per
// instance converged / not converged / a new cycle from r / |r|.
// ---------------------------------------------------------------------------
constexpr int kGDscal = 256;     // scalar slots per instance in g_dscal

struct GState {
    double R[(kMaxBasis + 1) * kMaxBasis];   // rotated columns, R[i * kMaxBasis + c]
    double Hc[kMaxBasis + 1];                // unrotated last column (rows 0..j+1)
    double cs[kMaxBasis], sn[kMaxBasis];
    double g[kMaxBasis + 1];
    double y[kMaxBasis];
    double gt, bnorm, beta, rt_prev, est, true_rel;
    int k, iters, restarts, status, done, pad;
};

// the step-j Givens update of every running instance (lane 0 of block r)
__global__ __launch_bounds__(64) void k_grp_givens(GState *__restrict__ st,
                                                   const double *__restrict__ dscal, int ds,
                                                   int *__restrict__ run, int *__restrict__ fin,
                                                   int j, int m, int maxit, double tol)
{
    const int r = blockIdx.x;
    if (threadIdx.x != 0 || !run[r]) return;
    GState &S = st[r];
    const double *d = dscal + (size_t)r * ds;
    const double *a = d + kRaw, *b = d + kRaw + j;
    const double rho = d[kOut], hj = d[kOut + 1], rt = d[kOut + 2];
    if (!(rho > 0.0) || !isfinite(rho) || !isfinite(hj) || !isfinite(rt)) {
        S.status = FMM_ERR_NUMERIC;
        S.done = 1;
        run[r] = 0;
        fin[r] = 0;
        return;
    }
    double *Hc = S.Hc;
    if (j == 0) {
        S.g[0] = S.beta * rho;              // r = beta u_0 = beta rho v_0
    } else {
        // column j - 1: the delayed correction, the committed rotations, its own
        for (int i = 0; i < j; ++i) Hc[i] += S.rt_prev * a[i];
        Hc[j] = S.rt_prev * rho;
        for (int i = 0; i + 1 < j; ++i) {
            const double x0 = Hc[i], x1 = Hc[i + 1];
            Hc[i] = S.cs[i] * x0 + S.sn[i] * x1;
            Hc[i + 1] = -S.sn[i] * x0 + S.cs[i] * x1;
        }
        const double x0 = Hc[j - 1], x1 = Hc[j];
        const double rr = hypot(x0, x1);
        S.cs[j - 1] = x0 / rr;
        S.sn[j - 1] = x1 / rr;
        for (int i = 0; i + 1 < j; ++i) S.R[i * kMaxBasis + j - 1] = Hc[i];
        S.R[(j - 1) * kMaxBasis + j - 1] = rr;
        S.g[j] = -S.sn[j - 1] * S.g[j - 1];
        S.g[j - 1] = S.cs[j - 1] * S.g[j - 1];
    }
    // column j: kept unrotated for the next step's correction, rotated for R
    for (int i = 0; i < j; ++i) Hc[i] = b[i];
    Hc[j] = hj;
    Hc[j + 1] = rt;
    double c[kMaxBasis + 1];
    for (int i = 0; i <= j + 1; ++i) c[i] = Hc[i];
    for (int i = 0; i < j; ++i) {
        const double x0 = c[i], x1 = c[i + 1];
        c[i] = S.cs[i] * x0 + S.sn[i] * x1;
        c[i + 1] = -S.sn[i] * x0 + S.cs[i] * x1;
    }
    const double rr = hypot(c[j], c[j + 1]);
    const double cst = c[j] / rr, snt = c[j + 1] / rr;
    for (int i = 0; i < j; ++i) S.R[i * kMaxBasis + j] = c[i];
    S.R[j * kMaxBasis + j] = rr;
    S.gt = cst * S.g[j];
    S.est = fabs(snt * S.g[j]) / S.bnorm;
    S.rt_prev = rt;
    S.iters += 1;
    if (S.est <= tol || rt == 0.0 || j + 1 == m || S.iters >= maxit) {
        S.k = j + 1;
        run[r] = 0;
        fin[r] = 1;
    }
}

// least squares of the cycle, y = R^-1 [g_0 .. g_{k-2}, gt], for the
// instances whose cycle ended
__global__ __launch_bounds__(64) void k_grp_lsq(GState *__restrict__ st, const int *__restrict__ fin)
{
    const int r = blockIdx.x;
    if (threadIdx.x != 0 || !fin[r]) return;
    GState &S = st[r];
    const int k = S.k;
    for (int i = k - 1; i >= 0; --i) {
        double acc = (i == k - 1) ? S.gt : S.g[i];
        for (int t = i + 1; t < k; ++t) acc -= S.R[i * kMaxBasis + t] * S.y[t];
        S.y[i] = acc / S.R[i * kMaxBasis + i];
    }
    S.restarts += 1;
}

// x_r += sum_{i < k_r} y_i Z_{r,i} for the instances whose cycle ended
__global__ __launch_bounds__(256) void k_grp_axpy(const GState *__restrict__ st,
                                                  const double *__restrict__ Z, int64_t ld,
                                                  double *__restrict__ x, Inst in, int64_t N)
{
    const int r = blockIdx.y;
    if (!inst_on(in, r)) return;
    const GState &S = st[r];
    const int k = S.k;
    Z += r * in.zs;
    x += r * in.xs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        double acc = x[e];
        for (int i = 0; i < k; ++i) acc = fma(S.y[i], Z[i * ld + e], acc);
        x[e] = acc;
    }
}

// norm of each flagged instance from its block partials (fixed order);
// which: 0 = |b| (bnorm), 1 = |r| (beta)
__global__ __launch_bounds__(256) void k_grp_norm(const double *__restrict__ part, int nblk,
                                                  GState *__restrict__ st, Inst in, int which)
{
    __shared__ double red[4];
    const int r = blockIdx.x;
    if (!inst_on(in, r)) return;
    const double *pi = part + r * in.ps;
    double a = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nblk; b += 256) a += pi[b];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double v = sqrt((red[0] + red[1]) + (red[2] + red[3]));
    if (which == 0) st[r].bnorm = v;
    else st[r].beta = v;
}

// after |b|: zero right-hand sides are solved by u = 0; the others start
// with the residual of their initial guess (fin marks them)
__global__ void k_grp_init(GState *__restrict__ st, int *__restrict__ run, int *__restrict__ fin,
                           int nr)
{
    const int r = blockIdx.x * 64 + threadIdx.x;
    if (r >= nr) return;
    GState &S = st[r];
    run[r] = 0;
    S.iters = S.restarts = 0;
    S.est = 1.0;
    S.true_rel = 1.0;
    if (!isfinite(S.bnorm)) {
        S.status = FMM_ERR_NUMERIC;
        S.done = 1;
        fin[r] = 0;
    } else if (S.bnorm == 0.0) {
        S.status = FMM_OK;
        S.true_rel = 0.0;
        S.done = 2;            // u = 0 is the solution (set by k_grp_zero)
        fin[r] = 0;
    } else {
        S.status = FMM_NOT_CONVERGED;
        S.done = 0;
        fin[r] = 1;
    }
}

__global__ __launch_bounds__(256) void k_grp_zero(const GState *__restrict__ st,
                                                  double *__restrict__ x, int64_t xs, int64_t N)
{
    const int r = blockIdx.y;
    if (st[r].done != 2) return;
    x += r * xs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256)
        x[e] = 0.0;
}

// after |r| of the instances whose cycle ended (fin): converged, out of
// iterations, or a new cycle (run)
__global__ void k_grp_cycle(GState *__restrict__ st, int *__restrict__ run, int *__restrict__ fin,
                            int nr, int maxit, double tol)
{
    const int r = blockIdx.x * 64 + threadIdx.x;
    if (r >= nr || !fin[r]) return;
    fin[r] = 0;
    GState &S = st[r];
    const double rel = S.beta / S.bnorm;
    S.true_rel = rel;
    if (!isfinite(S.beta)) {
        S.status = FMM_ERR_NUMERIC;
        S.done = 1;
    } else if (rel <= tol) {
        S.status = FMM_OK;
        S.done = 1;
    } else if (S.iters >= maxit) {
        S.status = FMM_NOT_CONVERGED;
        S.done = 1;
    } else {
        S.rt_prev = 0.0;
        run[r] = 1;
    }
}

// v_0 = r / |r| for the instances that start a cycle
__global__ __launch_bounds__(256) void k_grp_scale(const GState *__restrict__ st,
                                                   const double *__restrict__ w,
                                                   double *__restrict__ V, Inst in, int64_t N)
{
    const int r = blockIdx.y;
    if (!inst_on(in, r)) return;
    const double f = 1.0 / st[r].beta;
    w += r * in.xs;
    V += r * in.vs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256)
        V[e] = w[e] * f;
}

__global__ void k_grp_report(const GState *__restrict__ st, int *__restrict__ status, int nr)
{
    const int r = blockIdx.x * 64 + threadIdx.x;
    if (r < nr) status[r] = st[r].done ? st[r].status : 2;   // 2: still running
}

void release_group(fmm_plan *pl)
{
    void *ptrs[] = {pl->g_basis, pl->g_b, pl->g_x, pl->g_w, pl->g_part, pl->g_dscal, pl->g_state,
                    pl->g_flags};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (pl->g_host) (void)hipHostFree(pl->g_host);
    pl->g_basis = pl->g_b = pl->g_x = pl->g_w = pl->g_part = pl->g_dscal = nullptr;
    pl->g_state = nullptr;
    pl->g_flags = pl->g_host = nullptr;
    pl->g_cap = pl->g_m = 0;
}

static int ensure_group(fmm_plan *pl, int nr, int m)
{
    int st = ensure_rhs(pl, nr);
    if (st != FMM_OK) return st;
    if (pl->g_cap >= nr && pl->g_m == m) return FMM_OK;
    drop_step_graphs(pl);
    release_group(pl);
    const size_t N = (size_t)pl->n * pl->n;
    const int64_t ld = (int64_t)N + kBasisPad;
    pl->g_vs = (int64_t)(2 * m + 1) * ld;
    auto alloc = [&](void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
    if (!alloc((void **)&pl->g_basis, (size_t)nr * pl->g_vs * sizeof(double)) ||
        !alloc((void **)&pl->g_b, (size_t)nr * N * sizeof(double)) ||
        !alloc((void **)&pl->g_x, (size_t)nr * N * sizeof(double)) ||
        !alloc((void **)&pl->g_w, (size_t)nr * N * sizeof(double)) ||
        !alloc((void **)&pl->g_part, (size_t)nr * kPartRows * kRedBlocks * sizeof(double)) ||
        !alloc((void **)&pl->g_dscal, (size_t)nr * kGDscal * sizeof(double)) ||
        !alloc(&pl->g_state, (size_t)nr * sizeof(GState)) ||
        !alloc((void **)&pl->g_flags, (size_t)3 * nr * sizeof(int))) {
        release_group(pl);
        return fail(pl, FMM_ERR_ALLOC, "group solve workspace allocation failed");
    }
    FMM_HIP(pl, hipMemset(pl->g_state, 0, (size_t)nr * sizeof(GState)));
    FMM_HIP(pl, hipMemset(pl->g_flags, 0, (size_t)3 * nr * sizeof(int)));
    FMM_HIP(pl, hipHostMalloc((void **)&pl->g_host, (size_t)2 * nr * sizeof(int), hipHostMallocDefault));
    pl->g_cap = nr;
    pl->g_m = m;
    return FMM_OK;
}

// Resumable group FGMRES(m), driven like Fgmres: each issue_*() enqueues a
// chunk of GPU work ending with a copy of the run flags (or statuses) into
// pinned memory; advance() runs once that work has completed.
class GroupSolve {
  public:
    GroupSolve(fmm_plan *pl, int nr, const double *const *f, double *const *u,
               const gmres_params &prm, hipStream_t s, bool graphs)
        : pl_(pl), nr_(nr), f_(f), u_(u), tol_(prm.tol), m_(prm.restart), maxit_(prm.maxit), s_(s),
          graphs_(graphs)
    {
    }

    int begin()
    {
        int st = ensure_group(pl_, nr_, m_);
        if (st != FMM_OK) return st;
        // the captured launches carry the instance count and the solver
        // settings as arguments: other values need new graphs
        if (graphs_ && (pl_->g_graph_nr != nr_ || pl_->g_graph_maxit != maxit_ ||
                        pl_->g_graph_tol != tol_)) {
            drop_step_graphs(pl_);
            pl_->g_graph_nr = nr_;
            pl_->g_graph_maxit = maxit_;
            pl_->g_graph_tol = tol_;
        }
        n_ = (int)pl_->n;
        N_ = (int64_t)n_ * n_;
        ld_ = N_ + kBasisPad;
        ln_ = pl_->L + 3;
        ih2_ = 1.0 / (pl_->h * pl_->h);
        nblk_ = red_blocks(pl_, N_);
        S_ = static_cast<GState *>(pl_->g_state);
        run_ = pl_->g_flags;
        fin_ = pl_->g_flags + nr_;
        in_.vs = in_.zs = pl_->g_vs;
        in_.xs = N_;
        in_.ps = (int64_t)kPartRows * kRedBlocks;
        in_.ds = kGDscal;
        for (int r = 0; r < nr_; ++r) {
            FMM_HIP(pl_, hipMemcpyAsync(pl_->g_b + r * N_, f_[r], N_ * sizeof(double),
                                        hipMemcpyDeviceToDevice, s_));
            FMM_HIP(pl_, hipMemcpyAsync(pl_->g_x + r * N_, u_[r], N_ * sizeof(double),
                                        hipMemcpyDeviceToDevice, s_));
        }
        const dim3 gv(nblk_, nr_), gs((nr_ + 63) / 64);
        Inst all = in_;
        all.act = nullptr;
        hipLaunchKernelGGL(k_sumsq, gv, dim3(256), 0, s_, pl_->g_b, pl_->g_part, N_, all);
        hipLaunchKernelGGL(k_grp_norm, dim3(nr_), dim3(256), 0, s_, pl_->g_part, nblk_, S_, all, 0);
        hipLaunchKernelGGL(k_grp_init, gs, dim3(64), 0, s_, S_, run_, fin_, nr_);
        hipLaunchKernelGGL(k_grp_zero, gv, dim3(256), 0, s_, S_, pl_->g_x, N_, N_);
        cycle_tail();
        return copy_flags();
    }

    // the work chunk that just completed decides the next one
    int advance()
    {
        FMM_HIP(pl_, hipGetLastError());
        // every chunk is a step (at most maxit) or a cycle end (one per step
        // at most, plus the first): anything beyond that is an internal error
        if (++chunks_ > 2 * maxit_ + 4)
            return fail(pl_, FMM_ERR_DEVICE, "internal: group solve did not terminate");
        bool any = false;
        for (int r = 0; r < nr_; ++r) any = any || pl_->g_host[r] != 0;
        if (phase_ == CYCLE) {
            if (!any) {
                phase_ = DONE;
                return report();
            }
            j_ = 0;
            return issue_step();
        }
        if (phase_ == STEP) {
            if (any && j_ + 1 < m_) {
                ++j_;
                return issue_step();
            }
            return issue_end();
        }
        return FMM_OK;
    }

    bool done() const { return phase_ == DONE; }
    // after a chunk that ended a cycle: the status of instance r (2 while
    // it still runs), from the pinned copy
    bool cycle_ended() const { return phase_ == CYCLE || phase_ == DONE; }
    int host_status(int r) const { return pl_->g_host[nr_ + r]; }
    // statuses and results, valid once done() (and the stream has completed)
    int finish(gmres_result *res, int *status)
    {
        std::vector<GState> hs(nr_);
        FMM_HIP(pl_, hipMemcpy(hs.data(), S_, nr_ * sizeof(GState), hipMemcpyDeviceToHost));
        for (int r = 0; r < nr_; ++r) {
            FMM_HIP(pl_, hipMemcpyAsync(u_[r], pl_->g_x + r * N_, N_ * sizeof(double),
                                        hipMemcpyDeviceToDevice, s_));
            if (res) {
                res[r].iters = hs[r].iters;
                res[r].restarts = hs[r].restarts;
                res[r].est_rel_res = hs[r].est;
                res[r].true_rel_res = hs[r].true_rel;
            }
            if (status) status[r] = hs[r].status;
        }
        return FMM_OK;
    }

  private:
    enum Phase { CYCLE, STEP, DONE };

    // residual of the instances whose cycle ended, their verdicts, and v_0 of
    // those that go on
    void cycle_tail()
    {
        const dim3 gv(nblk_, nr_), gs((nr_ + 63) / 64);
        Inst fin = in_, run = in_;
        fin.act = fin_;
        run.act = run_;
        {
            StageTimer t(pl_, FMM_STAGE_STENCIL, s_);
            hipLaunchKernelGGL(k_residual<false>, gv, dim3(256), 0, s_, pl_->g_b, pl_->g_x, pl_->g_w,
                               pl_->g_part, n_, ln_, ih2_, Faces{nullptr, nullptr}, fin);
        }
        hipLaunchKernelGGL(k_grp_norm, dim3(nr_), dim3(256), 0, s_, pl_->g_part, nblk_, S_, fin, 1);
        hipLaunchKernelGGL(k_grp_cycle, gs, dim3(64), 0, s_, S_, run_, fin_, nr_, maxit_, tol_);
        hipLaunchKernelGGL(k_grp_scale, gv, dim3(256), 0, s_, S_, pl_->g_w, pl_->g_basis, run, N_);
        hipLaunchKernelGGL(k_grp_report, gs, dim3(64), 0, s_, S_, fin_ + nr_, nr_);
        phase_ = CYCLE;
    }

    // run flags (and after a cycle the statuses, which follow them in g_flags)
    int copy_flags()
    {
        const int cnt = phase_ == CYCLE ? 2 * nr_ : nr_;
        FMM_HIP(pl_, hipMemcpyAsync(pl_->g_host, run_, nr_ * sizeof(int), hipMemcpyDeviceToHost, s_));
        if (cnt > nr_)
            FMM_HIP(pl_, hipMemcpyAsync(pl_->g_host + nr_, fin_ + nr_, nr_ * sizeof(int),
                                        hipMemcpyDeviceToHost, s_));
        return FMM_OK;
    }

    int launch_step(int j)
    {
        double *V = pl_->g_basis, *Z = pl_->g_basis + (size_t)(m_ + 1) * ld_;
        double *uj = V + (size_t)j * ld_, *zj = Z + (size_t)j * ld_;
        int st = precond_apply_rhs(pl_, uj, zj, nr_, pl_->g_vs, run_, s_);
        if (st != FMM_OK) return st;
        StageTimer ta(pl_, FMM_STAGE_ARNOLDI, s_);
        Inst run = in_;
        run.act = run_;
        const dim3 gv(nblk_, nr_);
        launch_arnoldi_dots<false>(j, gv, s_, zj, V, ld_, pl_->g_part, n_, ln_, ih2_,
                                   Faces{nullptr, nullptr}, run);
        hipLaunchKernelGGL(k_arnoldi_coef, dim3(nr_), dim3(1024), 0, s_, pl_->g_part, nblk_,
                           pl_->g_dscal, j, run);
        hipLaunchKernelGGL(k_grp_givens, dim3(nr_), dim3(64), 0, s_, S_, pl_->g_dscal, kGDscal, run_,
                           fin_, j, m_, maxit_, tol_);
        launch_arnoldi_update<false>(j, gv, s_, zj, V, ld_, pl_->g_dscal + kCoef, n_, ln_, ih2_,
                                     Faces{nullptr, nullptr}, run);
        ta.stop();
        return copy_flags();
    }

    int launch_end()
    {
        const dim3 gv(nblk_, nr_), gs((nr_ + 63) / 64);
        Inst fin = in_;
        fin.act = fin_;
        hipLaunchKernelGGL(k_grp_lsq, dim3(nr_), dim3(64), 0, s_, S_, fin_);
        {
            StageTimer ta(pl_, FMM_STAGE_ARNOLDI, s_);
            hipLaunchKernelGGL(k_grp_axpy, gv, dim3(256), 0, s_, S_,
                               pl_->g_basis + (size_t)(m_ + 1) * ld_, ld_, pl_->g_x, fin, N_);
        }
        cycle_tail();
        return copy_flags();
    }

    // runs fn directly, or from the graph it was captured into the first time
    template <class F>
    int replay(hipGraphExec_t &ex, F fn)
    {
        if (!graphs_ || pl_->prof_mask) return fn();
        if (!ex) {
            hipGraph_t gr = nullptr;
            FMM_HIP(pl_, hipStreamBeginCapture(s_, hipStreamCaptureModeRelaxed));
            const int st = fn();
            const hipError_t ec = hipStreamEndCapture(s_, &gr);
            if (st != FMM_OK) {
                if (gr) (void)hipGraphDestroy(gr);
                return st;
            }
            FMM_HIP(pl_, ec);
            const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            FMM_HIP(pl_, ei);
        }
        FMM_HIP(pl_, hipGraphLaunch(ex, s_));
        return FMM_OK;
    }

    int issue_step()
    {
        phase_ = STEP;
        if ((int)pl_->g_step_exec.size() < m_) pl_->g_step_exec.resize(m_, nullptr);
        const int j = j_;
        return replay(pl_->g_step_exec[j], [&]() { return launch_step(j); });
    }

    // (the phase is set here: a replayed graph does not run launch_end)
    int issue_end()
    {
        phase_ = CYCLE;
        return replay(pl_->g_end_exec, [&]() { return launch_end(); });
    }

    int report() { return FMM_OK; }

    fmm_plan *pl_;
    int nr_;
    const double *const *f_;
    double *const *u_;
    double tol_;
    int m_, maxit_;
    hipStream_t s_;
    bool graphs_;
    Phase phase_ = CYCLE;
    int chunks_ = 0;
    int j_ = 0, n_ = 0, ln_ = 0, nblk_ = 1;
    int64_t N_ = 0, ld_ = 0;
    double ih2_ = 0.0;
    GState *S_ = nullptr;
    int *run_ = nullptr, *fin_ = nullptr;
    Inst in_;
};

int gmres_solve_group(fmm_plan *pl, int nr, const double *const *f, double *const *u,
                      const gmres_params *prm, gmres_result *res, bool graphs, hipStream_t s)
{
    GroupSolve g(pl, nr, f, u, *prm, s, graphs);
    int st = g.begin();
    while (st == FMM_OK && !g.done()) {
        FMM_HIP(pl, hipStreamSynchronize(s));
        st = g.advance();
    }
    if (st != FMM_OK) return st;
    std::vector<int> status(nr);
    st = g.finish(res, status.data());
    if (st != FMM_OK) return st;
    FMM_HIP(pl, hipStreamSynchronize(s));
    int overall = FMM_OK;
    for (int r = 0; r < nr; ++r) {
        if (status[r] < 0) return fail(pl, status[r], "a group instance failed (non-finite values)");
        if (status[r] != FMM_OK) overall = FMM_NOT_CONVERGED;
    }
    return overall;
}


// Batched solves by groups: instances whose plans describe the same problem
// (grid size, p, precision, theta, self term, boundary correction) are
// solved together, at most kMaxRhsChunk per group, each group on the plan of
// its first instance (that plan's workspace holds the whole group) and on
// that plan's stream.  A host loop polls the groups' events and advances
// whichever group's last chunk of work has completed, so groups of
// different sizes overlap on the GPU.
static int gmres_solve_batch_grouped(fmm_plan *const *plans, int count, const double *const *f,
                                     double *const *u, const gmres_params *prm, gmres_result *res,
                                     double *elapsed_ms, bool graphs, hipStream_t caller)
{
    struct Group {
        fmm_plan *pl;
        std::vector<int> idx;
        std::vector<const double *> f;
        std::vector<double *> u;
        std::vector<char> seen;
        std::unique_ptr<GroupSolve> gs;
        bool fin = false;
    };
    std::vector<Group> groups;
    auto same = [](const fmm_plan *a, const fmm_plan *b) {
        return a->n == b->n && a->p == b->p && a->prec == b->prec && a->bem == b->bem &&
               a->theta == b->theta && a->self_eps == b->self_eps;
    };
    for (int i = 0; i < count; ++i) {
        Group *g = nullptr;
        for (auto &c : groups)
            if (same(c.pl, plans[i]) && (int)c.idx.size() < kMaxRhsChunk) g = &c;
        if (!g) {
            groups.emplace_back();
            g = &groups.back();
            g->pl = plans[i];
        }
        g->idx.push_back(i);
        g->f.push_back(f[i]);
        g->u.push_back(u[i]);
    }
    hipEvent_t start = nullptr;
    fmm_plan *p0 = plans[0];
    FMM_HIP(p0, hipEventCreateWithFlags(&start, hipEventDisableTiming));
    FMM_HIP(p0, hipEventRecord(start, caller));
    int st = FMM_OK;
    for (auto &g : groups) {
        fmm_plan *pl = g.pl;
        if (st == FMM_OK && !pl->bstream && hipStreamCreateWithFlags(&pl->bstream, hipStreamNonBlocking) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "stream creation failed");
        if (st == FMM_OK && !pl->bevent && hipEventCreateWithFlags(&pl->bevent, hipEventDisableTiming) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "event creation failed");
        if (st == FMM_OK && hipStreamWaitEvent(pl->bstream, start, 0) != hipSuccess)
            st = fail(pl, FMM_ERR_DEVICE, "stream wait failed");
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (auto &g : groups) {
        if (st != FMM_OK) break;
        g.seen.assign(g.idx.size(), 0);
        g.gs.reset(new GroupSolve(g.pl, (int)g.idx.size(), g.f.data(), g.u.data(), *prm, g.pl->bstream,
                                  graphs));
        st = g.gs->begin();
        if (st == FMM_OK && hipEventRecord(g.pl->bevent, g.pl->bstream) != hipSuccess)
            st = fail(g.pl, FMM_ERR_DEVICE, "event record failed");
    }
    fmm_plan *failed = nullptr;
    int active = (int)groups.size();
    while (st == FMM_OK && active > 0) {
        bool moved = false;
        for (auto &g : groups) {
            if (g.fin || st != FMM_OK) continue;
            const hipError_t q = hipEventQuery(g.pl->bevent);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                st = fail(g.pl, FMM_ERR_DEVICE, hipGetErrorString(q));
                failed = g.pl;
                break;
            }
            moved = true;
            if (g.gs->cycle_ended() && elapsed_ms) {
                const double ms = std::chrono::duration<double, std::milli>(
                                      std::chrono::steady_clock::now() - t0).count();
                for (size_t r = 0; r < g.idx.size(); ++r)
                    if (!g.seen[r] && g.gs->host_status((int)r) != 2) {
                        g.seen[r] = 1;
                        elapsed_ms[g.idx[r]] = ms;
                    }
            }
            st = g.gs->advance();
            if (st != FMM_OK) {
                failed = g.pl;
                break;
            }
            if (g.gs->done()) {
                std::vector<gmres_result> rr(g.idx.size());
                std::vector<int> stat(g.idx.size());
                st = g.gs->finish(rr.data(), stat.data());
                if (st != FMM_OK) {
                    failed = g.pl;
                    break;
                }
                for (size_t r = 0; r < g.idx.size(); ++r) {
                    if (res) res[g.idx[r]] = rr[r];
                    if (stat[r] < 0 && st == FMM_OK) {
                        st = fail(g.pl, stat[r], "a batched instance met non-finite values");
                        failed = g.pl;
                    }
                }
                g.fin = true;
                --active;
            }
            if (hipEventRecord(g.pl->bevent, g.pl->bstream) != hipSuccess && st == FMM_OK) {
                st = fail(g.pl, FMM_ERR_DEVICE, "event record failed");
                failed = g.pl;
            }
        }
        if (!moved) std::this_thread::yield();
    }
    int overall = FMM_OK;
    for (auto &g : groups) {
        if (g.pl->bevent) {
            (void)hipEventRecord(g.pl->bevent, g.pl->bstream);
            (void)hipStreamWaitEvent(caller, g.pl->bevent, 0);
        }
        if (st != FMM_OK) (void)hipStreamSynchronize(g.pl->bstream);
    }
    (void)hipEventDestroy(start);
    if (st != FMM_OK) {
        if (failed && failed != p0) p0->err = failed->err;
        return st;
    }
    if (res)
        for (int i = 0; i < count; ++i)
            if (!(res[i].true_rel_res <= prm->tol)) overall = FMM_NOT_CONVERGED;
    return overall;
}

int gmres_solve_batch(fmm_plan *const *plans, int count, const double *const *f, double *const *u,
                      const gmres_params *prm, gmres_result *res, double *elapsed_ms, bool graphs,
                      bool separate, hipStream_t caller)
{
    if (separate)
        return gmres_solve_batch_separate(plans, count, f, u, prm, res, elapsed_ms, graphs, caller);
    for (int i = 0; i < count; ++i)
        if (plans[i]->prof_mask) graphs = false;
    return gmres_solve_batch_grouped(plans, count, f, u, prm, res, elapsed_ms, graphs, caller);
}

// Tunes the block count of the Krylov vector kernels for this plan's grid:
// times sweep A and B of an Arnoldi step (j = 4) for each candidate (the
// fastest of three calls, over three rounds that visit the candidates in
// turn) and keeps the fastest (small grids want more blocks than
// elements / 1024).
int tune_vector_blocks(fmm_plan *pl, hipStream_t s, int *chosen)
{
    int st = ensure_krylov(pl, 8);
    if (st != FMM_OK) return st;
    const int n = (int)pl->n, ln = pl->L + 3;
    const int64_t N = (int64_t)n * n;
    const double ih2 = 1.0 / (pl->h * pl->h);
    const int cands[] = {64, 128, 256, 512, 1024, 2048, 4096};
    hipEvent_t e0, e1;
    FMM_HIP(pl, hipEventCreate(&e0));
    FMM_HIP(pl, hipEventCreate(&e1));
    // a finite basis to sweep over (values do not affect the timing)
    hipLaunchKernelGGL(k_scale, dim3(256), dim3(256), 0, s, pl->V, pl->V, nullptr, 0.0, pl->ldb * 6);
    hipLaunchKernelGGL(k_scale, dim3(256), dim3(256), 0, s, pl->Z, pl->Z, nullptr, 0.0, N);
    constexpr int NC = sizeof(cands) / sizeof(cands[0]);
    float cand_ms[NC];
    for (int i = 0; i < NC; ++i) cand_ms[i] = 1e30f;
    for (int round = 0; round < 3; ++round)
        for (int i = 0; i < NC; ++i) {
            const int c = cands[i];
            if ((int64_t)c * 256 > 4 * N && c > 64) continue;   // under 4 elements per thread
            const int nb = c > kRedBlocks ? kRedBlocks : c;
            for (int rep = 0; rep < 4; ++rep) {
                FMM_HIP(pl, hipEventRecord(e0, s));
                launch_arnoldi_dots<false>(4, dim3(nb), s, pl->Z, pl->V, pl->ldb, pl->partial, n, ln, ih2,
                                           Faces{nullptr, nullptr});
                launch_arnoldi_update<false>(4, dim3(nb), s, pl->Z, pl->V, pl->ldb, pl->dscal + kCoef, n,
                                             ln, ih2, Faces{nullptr, nullptr});
                FMM_HIP(pl, hipEventRecord(e1, s));
                FMM_HIP(pl, hipEventSynchronize(e1));
                float t = 0.0f;
                FMM_HIP(pl, hipEventElapsedTime(&t, e0, e1));
                if (rep > 0) cand_ms[i] = std::min(cand_ms[i], t);
            }
        }
    float best_ms = 1e30f;
    int best = red_blocks(nullptr, N);
    for (int i = 0; i < NC; ++i)
        if (cand_ms[i] < best_ms) {
            best_ms = cand_ms[i];
            best = cands[i] > kRedBlocks ? kRedBlocks : cands[i];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (pl->vec_blocks != best) drop_step_graphs(pl);
    pl->vec_blocks = best;
    if (chosen) *chosen = best;
    return FMM_OK;
}

}  // namespace fmmprec
