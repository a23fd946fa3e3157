// Krylov solver around the FMM-BEM preconditioner: the 5-point stencil
// (Sec. 2.1, eq. axb) and right-preconditioned FGMRES(m) with classical
// Gram-Schmidt applied twice (GMRES is the Krylov method the paper cites in
// Sec. 1; right preconditioning as in Sec. 3.1).
//
// Every vector kernel is HBM bound.  The Arnoldi step is fused into three
// passes over the basis:
//   1. w = A z_j and the partial dots V^T w           (stencil + GEMV-T)
//   2. w -= V h1 and the partial dots V^T w           (GEMV + GEMV-T)
//   3. w -= V h2 and the partial sum of w^2           (GEMV + norm)
// followed by v_{j+1} = w / ||w||.  Reductions are two-stage with a fixed
// order (no atomics), so repeated solves are bitwise reproducible.  One
// small device-to-host copy per inner iteration feeds the Givens rotations
// on the host.
#include <cmath>
#include <vector>

#include "fmm_internal.h"

namespace fmmprec {

constexpr int kMaxBasis = 32;   // restart <= 32: at most 32 basis vectors in a dot
constexpr int kRedBlocks = 4096;  // partial sums per reduction (coefficient-major)

// layout of plan->dscal (device) / plan->hpin (host mirror)
constexpr int kH1 = 0, kHsum = 32, kNrm = 64, kH2 = 96, kScal = 128;

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

__device__ __forceinline__ double stencil_at(const double *__restrict__ v, int64_t e, int n)
{
    const int i = (int)(e % n), j = (int)(e / n);
    double c = 4.0 * v[e];
    if (i > 0) c -= v[e - 1];
    if (i < n - 1) c -= v[e + 1];
    if (j > 0) c -= v[e - n];
    if (j < n - 1) c -= v[e + n];
    return c;
}

// block-level sum of NV per-thread values into part[i * kRedBlocks + blockIdx.x]
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], int nv, double *part)
{
    __shared__ double red[4][kMaxBasis];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) {
            double a = acc[i];
            for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
            if (lane == 0) red[wv][i] = a;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv)
        part[(size_t)threadIdx.x * kRedBlocks + blockIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// w = A z (scaled by 1/h^2) and partial dots V_i . w, i < NV
template <int NV>
__global__ __launch_bounds__(256) void k_stencil_dots(const double *__restrict__ z,
                                                      double *__restrict__ w,
                                                      const double *__restrict__ V, int64_t ldv,
                                                      double *__restrict__ part, int n, double ih2)
{
    const int64_t N = (int64_t)n * n;
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        double vv[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) vv[i] = V[i * ldv + e];
        const double we = stencil_at(z, e, n) * ih2;
        w[e] = we;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = fma(vv[i], we, acc[i]);
    }
    block_reduce_store<NV>(acc, NV, part);
}

// w -= sum_i h_i V_i; then partial dots V_i . w (MODE 0) or partial w.w (MODE 1)
template <int NV, int MODE>
__global__ __launch_bounds__(256) void k_update(const double *__restrict__ V, int64_t ldv,
                                                double *__restrict__ w,
                                                const double *__restrict__ hc,
                                                double *__restrict__ part, int64_t N)
{
    constexpr int NA = MODE == 0 ? NV : 1;
    double acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.0;
    double hv[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hv[i] = hc[i];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        double vv[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) vv[i] = V[i * ldv + e];
        double we = w[e];
#pragma unroll
        for (int i = 0; i < NV; ++i) we = fma(-hv[i], vv[i], we);
        w[e] = we;
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < NA; ++i) acc[i] = fma(vv[i], we, acc[i]);
        } else {
            acc[0] = fma(we, we, acc[0]);
        }
    }
    block_reduce_store<NA>(acc, NA, part);
}

#define KRY_NV_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

static void launch_stencil_dots(int nv, dim3 g, hipStream_t s, const double *z, double *w,
                                const double *V, int64_t ldv, double *part, int n, double ih2)
{
    switch (nv) {
#define X(k) case k: hipLaunchKernelGGL(k_stencil_dots<k>, g, dim3(256), 0, s, z, w, V, ldv, part, n, ih2); break;
        KRY_NV_CASES(X)
#undef X
    }
}

static void launch_update(int nv, int mode, dim3 g, hipStream_t s, const double *V, int64_t ldv,
                          double *w, const double *hc, double *part, int64_t N)
{
    if (mode == 0) {
        switch (nv) {
#define X(k) case k: hipLaunchKernelGGL((k_update<k, 0>), g, dim3(256), 0, s, V, ldv, w, hc, part, N); break;
            KRY_NV_CASES(X)
#undef X
        }
    } else {
        switch (nv) {
#define X(k) case k: hipLaunchKernelGGL((k_update<k, 1>), g, dim3(256), 0, s, V, ldv, w, hc, part, N); break;
            KRY_NV_CASES(X)
#undef X
        }
    }
}

// r = b - A x, partial r.r
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ b,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ r,
                                                  double *__restrict__ part, int n, double ih2)
{
    const int64_t N = (int64_t)n * n;
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        const double re = b[e] - stencil_at(x, e, n) * ih2;
        r[e] = re;
        acc[0] = fma(re, re, acc[0]);
    }
    block_reduce_store<1>(acc, 1, part);
}

// partial v.v
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ v,
                                               double *__restrict__ part, int64_t N)
{
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256)
        acc[0] = fma(v[e], v[e], acc[0]);
    block_reduce_store<1>(acc, 1, part);
}

// out[i] = sum_b part[i][b] (+ add[i]); mode 1: out[i] = sqrt(sum); out2, if
// given, also receives the plain sum.  One block per coefficient i; the
// summation order is fixed.
__global__ __launch_bounds__(256) void k_finish(const double *__restrict__ part, int nblk,
                                                double *__restrict__ out,
                                                const double *__restrict__ add,
                                                double *__restrict__ out2, int mode)
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
    if (threadIdx.x == 0) {
        const double sum = (red[0] + red[1]) + (red[2] + red[3]);
        if (mode == 1) {
            out[i] = sqrt(sum);
        } else {
            if (out2) out2[i] = sum;
            out[i] = add ? sum + add[i] : sum;
        }
    }
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

static int red_blocks(int64_t N)
{
    int64_t b = (N + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    return (int)b;
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
    int st = grid_volume_fmm(pl, r, h2, z, need_ring ? pl->phi_ring : nullptr, s);
    if (st != FMM_OK) return st;
    if (phi_ring)
        FMM_HIP(pl, hipMemcpyAsync(phi_ring, pl->phi_ring, 4 * (size_t)pl->n * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
    if (pl->bem) {
        st = bem_apply(pl, sigma, s);
        if (st != FMM_OK) return st;
        st = grid_ring_source_fmm(pl, z, s);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

static int ensure_krylov(fmm_plan *pl, int m)
{
    if (pl->kry_m >= m) return FMM_OK;
    const size_t N = (size_t)pl->n * pl->n;
    if (pl->V) { hipFree(pl->V); pl->V = nullptr; }
    if (pl->Z) { hipFree(pl->Z); pl->Z = nullptr; }
    if (!pl->w) FMM_HIP(pl, hipMalloc(&pl->w, N * sizeof(double)));
    if (!pl->b) FMM_HIP(pl, hipMalloc(&pl->b, N * sizeof(double)));
    if (!pl->partial) FMM_HIP(pl, hipMalloc(&pl->partial, (size_t)kRedBlocks * kMaxBasis * sizeof(double)));
    if (!pl->dscal) FMM_HIP(pl, hipMalloc(&pl->dscal, 256 * sizeof(double)));
    if (!pl->hpin) FMM_HIP(pl, hipHostMalloc((void **)&pl->hpin, 256 * sizeof(double), hipHostMallocDefault));
    hipError_t e1 = hipMalloc(&pl->V, (size_t)(m + 1) * N * sizeof(double));
    if (e1 != hipSuccess) return fail(pl, FMM_ERR_ALLOC, "Krylov basis allocation failed");
    hipError_t e2 = hipMalloc(&pl->Z, (size_t)m * N * sizeof(double));
    if (e2 != hipSuccess) return fail(pl, FMM_ERR_ALLOC, "Krylov basis allocation failed");
    pl->kry_m = m;
    return FMM_OK;
}

// reduce partials of a norm kernel into dscal[slot] = sqrt(sum) and fetch it
static int fetch_norm(fmm_plan *pl, int nblk, int slot, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, pl->partial, nblk, pl->dscal + slot,
                       nullptr, nullptr, 1);
    FMM_HIP(pl, hipMemcpyAsync(pl->hpin + slot, pl->dscal + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    FMM_HIP(pl, hipStreamSynchronize(s));
    *out = pl->hpin[slot];
    return FMM_OK;
}

int gmres_solve(fmm_plan *pl, const double *f, const double *g, double *u, const gmres_params *prm,
                gmres_result *res, hipStream_t s)
{
    const double tol = prm->tol;
    const int m = prm->restart, maxit = prm->maxit;
    int st = ensure_krylov(pl, m);
    if (st != FMM_OK) return st;
    const int n = (int)pl->n;
    const int64_t N = (int64_t)n * n;
    const double ih2 = 1.0 / (pl->h * pl->h);
    const int nblk = red_blocks(N);
    const dim3 gv(nblk), bv(256);

    hipLaunchKernelGGL(k_make_rhs, gv, bv, 0, s, f, g, pl->b, n, ih2);
    hipLaunchKernelGGL(k_sumsq, gv, bv, 0, s, pl->b, pl->partial, N);
    double bnorm = 0.0;
    if ((st = fetch_norm(pl, nblk, kScal, &bnorm, s)) != FMM_OK) return st;
    gmres_result r{};
    if (!std::isfinite(bnorm)) return fail(pl, FMM_ERR_NUMERIC, "right-hand side is not finite");
    if (bnorm == 0.0) {
        FMM_HIP(pl, hipMemsetAsync(u, 0, N * sizeof(double), s));
        FMM_HIP(pl, hipStreamSynchronize(s));
        if (res) *res = r;
        return FMM_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gg(m + 1), y(m);
    int iters = 0, status = FMM_NOT_CONVERGED;
    double est = 1.0;
    for (;;) {
        // true residual of the current iterate
        {
            StageTimer t(pl, FMM_STAGE_STENCIL, s);
            hipLaunchKernelGGL(k_residual, gv, bv, 0, s, pl->b, u, pl->w, pl->partial, n, ih2);
        }
        double beta = 0.0;
        if ((st = fetch_norm(pl, nblk, kScal, &beta, s)) != FMM_OK) return st;
        if (!std::isfinite(beta)) return fail(pl, FMM_ERR_NUMERIC, "residual is not finite");
        r.true_rel_res = beta / bnorm;
        if (beta / bnorm <= tol) { status = FMM_OK; break; }
        if (iters >= maxit) { status = FMM_NOT_CONVERGED; break; }
        hipLaunchKernelGGL(k_scale, gv, bv, 0, s, pl->w, pl->V, nullptr, 1.0 / beta, N);
        std::fill(gg.begin(), gg.end(), 0.0);
        gg[0] = beta;
        int k = 0;
        for (int j = 0; j < m && iters < maxit; ++j) {
            double *vj = pl->V + (size_t)j * N, *zj = pl->Z + (size_t)j * N;
            if ((st = precond_apply_one(pl, vj, zj, nullptr, nullptr, s)) != FMM_OK) return st;
            const int nv = j + 1;
            StageTimer ta(pl, FMM_STAGE_ARNOLDI, s);
            // pass 1: w = A z_j, h1 = V^T w
            launch_stencil_dots(nv, gv, s, zj, pl->w, pl->V, N, pl->partial, n, ih2);
            hipLaunchKernelGGL(k_finish, dim3(nv), dim3(256), 0, s, pl->partial, nblk, pl->dscal + kH1,
                               nullptr, nullptr, 0);
            // pass 2: w -= V h1, h2 = V^T w, hsum = h1 + h2
            launch_update(nv, 0, gv, s, pl->V, N, pl->w, pl->dscal + kH1, pl->partial, N);
            hipLaunchKernelGGL(k_finish, dim3(nv), dim3(256), 0, s, pl->partial, nblk, pl->dscal + kHsum,
                               pl->dscal + kH1, pl->dscal + kH2, 0);
            // pass 3: w -= V h2, ||w||
            launch_update(nv, 1, gv, s, pl->V, N, pl->w, pl->dscal + kH2, pl->partial, N);
            hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, pl->partial, nblk, pl->dscal + kNrm,
                               nullptr, nullptr, 1);
            hipLaunchKernelGGL(k_scale, gv, bv, 0, s, pl->w, pl->V + (size_t)(j + 1) * N, pl->dscal + kNrm, 0.0, N);
            ta.stop();
            FMM_HIP(pl, hipMemcpyAsync(pl->hpin + kHsum, pl->dscal + kHsum, 33 * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
            FMM_HIP(pl, hipStreamSynchronize(s));
            FMM_HIP(pl, hipGetLastError());
            const double hn = pl->hpin[kNrm];
            if (!std::isfinite(hn)) return fail(pl, FMM_ERR_NUMERIC, "Arnoldi produced a non-finite norm");
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = pl->hpin[kHsum + i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a, c);
            cs[j] = a / rr;
            sn[j] = c / rr;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gg[j + 1] = -sn[j] * gg[j];
            gg[j] = cs[j] * gg[j];
            ++iters;
            k = j + 1;
            est = std::fabs(gg[j + 1]) / bnorm;
            if (est <= tol || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double sacc = gg[i];
            for (int t = i + 1; t < k; ++t) sacc -= H[(size_t)i * m + t] * y[t];
            y[i] = sacc / H[(size_t)i * m + i];
        }
        Coef cy{};
        for (int i = 0; i < k; ++i) cy.c[i] = y[i];
        hipLaunchKernelGGL(k_axpy_multi, gv, bv, 0, s, pl->Z, N, k, cy, u, N);
        r.restarts++;
    }
    r.iters = iters;
    r.est_rel_res = est;
    FMM_HIP(pl, hipGetLastError());
    if (res) *res = r;
    return status;
}

}  // namespace fmmprec
