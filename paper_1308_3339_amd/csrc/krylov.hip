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
// above this multiple of the tolerance (one more step cannot reach it)
constexpr double kSpecMargin = 1e3;

__global__ __launch_bounds__(256) void k_stencil(const double *__restrict__ v,
                                                 double *__restrict__ w, int n, double ih2)
{
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
                                                      double ih2, Faces fc)
{
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
                                                       double *__restrict__ d, int nj)
{
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
                                                        int ln, double ih2, Faces fc)
{
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
                                int64_t ldv, double *part, int n, int ln, double ih2, Faces fc)
{
    switch (nj) {
#define X(k) case k: hipLaunchKernelGGL((k_arnoldi_dots<k, VAR>), g, dim3(256), 0, s, z, V, ldv, part, n, ln, ih2, fc); break;
        KRY_NJ_CASES(X)
#undef X
    }
}

template <bool VAR>
static void launch_arnoldi_update(int nj, dim3 g, hipStream_t s, const double *z, double *V,
                                  int64_t ldv, const double *cf, int n, int ln, double ih2, Faces fc)
{
    switch (nj) {
#define X(k) case k: hipLaunchKernelGGL((k_arnoldi_update<k, VAR>), g, dim3(256), 0, s, z, V, ldv, cf, n, ln, ih2, fc); break;
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
                                                  double ih2, Faces fc)
{
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
                                               double *__restrict__ part, int64_t N)
{
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

int stencil_apply(fmm_plan *pl, const double *v, double *w, hipStream_t s)
{
    const int n = (int)pl->n;
    const double ih2 = 1.0 / (pl->h * pl->h);
    StageTimer t(pl, FMM_STAGE_STENCIL, s);
    hipLaunchKernelGGL(k_stencil, dim3((n + 63) / 64, (n + 3) / 4), dim3(256), 0, s, v, w, n, ih2);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int precond_apply_one(fmm_plan *pl, const double *r, double *z, double *phi_ring, double *sigma,
                      hipStream_t s)
{
    const double h2 = pl->h * pl->h;
    const bool need_ring = pl->bem || phi_ring;
    int st = grid_volume_fmm(pl, r, h2, z, need_ring ? pl->phi_ring : nullptr, pl->bem != 0, s);
    if (st != FMM_OK) return st;
    if (phi_ring)
        FMM_HIP(pl, hipMemcpyAsync(phi_ring, pl->phi_ring, 4 * (size_t)pl->n * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
    if (pl->bem) {
        st = bem_apply(pl, sigma, s);
        if (st != FMM_OK) return st;
        st = grid_ring_source_fmm(pl, z, true, sigma, s);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

void drop_step_graphs(fmm_plan *pl)
{
    for (auto &ex : pl->step_exec)
        if (ex) (void)hipGraphExecDestroy(ex);
    pl->step_exec.clear();
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
        hipLaunchKernelGGL(k_sumsq, dim3(nblk_), dim3(256), 0, s_, pl_->b, pl_->partial, N_);
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
                                   pl_->partial, n_, ln_, ih2_, fc_);
            else
                hipLaunchKernelGGL(k_residual<false>, dim3(nblk_), dim3(256), 0, s_, pl_->b, u_, pl_->w,
                                   pl_->partial, n_, ln_, ih2_, fc_);
        }
        phase_ = RES;
        return fetch_scalar();
    }

    // the launches of Arnoldi step j (identical on every call, so capturable)
    // with spec: step j_ + 1 now, if an estimate of est leaves it certainly needed
    int issue_ahead(double est)
    {
        if (!spec_ || j_ + 1 >= m_ || iters_ + 2 > maxit_ || !(est > tol_ * kSpecMargin)) return FMM_OK;
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
                           pl_->dscal, j);
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
        est_ = std::fabs(gg_[j + 1]) / bnorm_;
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

int gmres_solve_batch(fmm_plan *const *plans, int count, const double *const *f, double *const *u,
                      const gmres_params *prm, gmres_result *res, double *elapsed_ms, bool graphs,
                      hipStream_t caller)
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

// Tunes the block count of the Krylov vector kernels for this plan's grid:
// times sweep A and B of an Arnoldi step (j = 4) for each candidate and
// keeps the fastest (small grids want more blocks than elements / 1024).
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
    float best_ms = 1e30f;
    int best = red_blocks(nullptr, N);
    for (int c : cands) {
        if ((int64_t)c * 256 > 4 * N && c > 64) continue;   // under 4 elements per thread
        const int nb = c > kRedBlocks ? kRedBlocks : c;
        float ms = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {
            FMM_HIP(pl, hipEventRecord(e0, s));
            launch_arnoldi_dots<false>(4, dim3(nb), s, pl->Z, pl->V, pl->ldb, pl->partial, n, ln, ih2,
                                       Faces{nullptr, nullptr});
            launch_arnoldi_update<false>(4, dim3(nb), s, pl->Z, pl->V, pl->ldb, pl->dscal + kCoef, n, ln,
                                         ih2, Faces{nullptr, nullptr});
            FMM_HIP(pl, hipEventRecord(e1, s));
            FMM_HIP(pl, hipEventSynchronize(e1));
            float t = 0.0f;
            FMM_HIP(pl, hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) ms += t;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = nb;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (pl->vec_blocks != best) drop_step_graphs(pl);
    pl->vec_blocks = best;
    if (chosen) *chosen = best;
    return FMM_OK;
}

}  // namespace fmmprec
