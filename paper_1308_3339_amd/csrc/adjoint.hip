// Differentiation support for the grid solve: the Gaussian-bump source model
// of the differentiation workload and the gradients of a scalar loss with
// respect to its parameters.  With u = A^{-1} f (A the symmetric 5-point
// matrix of Sec. 2.1), the adjoint dL/df = A^{-1} dL/du is one more
// preconditioned solve; these kernels carry dL/df on to the bump centres,
// widths and amplitudes:
//   f_i    = sum_k a_k e_ik,   e_ik = exp(-|x_i - c_k|^2 / (2 w_k^2))
//   dL/dc_k = a_k / w_k^2 sum_i g_i e_ik (x_i - c_k)
//   dL/dw_k = a_k / w_k^3 sum_i g_i e_ik |x_i - c_k|^2
//   dL/da_k = sum_i g_i e_ik
// Both kernels are HBM bound (one or two sweeps over the grid); the sums are
// two-stage with a fixed order, so results are bitwise reproducible.
#include <cmath>
#include <mutex>

#include "fmm_internal.h"

namespace fmmprec {

constexpr int kBumpMax = 256;        // bumps per call
constexpr int kBumpBlocks = 128;     // partial sums per (bump, quantity)

// Workspace of the allocation-free gradient entry point: the block partials
// of up to kBumpMax bumps, resident on every device the library runs on
// until the process ends (1 MiB each).  Host code never passes the array's
// name to a kernel: it takes the device address from hipGetSymbolAddress,
// once per device, and keeps it in g_scratch_addr.
constexpr int kScratchDoubles = kBumpMax * 4 * kBumpBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_addr[kMaxDevices] = {};

struct BumpParams {
    const double *cx, *cy, *w, *a;
};

// f_i for every interior node; bump parameters are block-uniform (LDS)
__global__ __launch_bounds__(256) void k_bumps_eval(BumpParams bp, int K, double *__restrict__ f,
                                                    int n, int ln, double h)
{
    __shared__ double scx[kBumpMax], scy[kBumpMax], sc[kBumpMax], sa[kBumpMax];
    for (int k = threadIdx.x; k < K; k += 256) {
        scx[k] = bp.cx[k];
        scy[k] = bp.cy[k];
        sc[k] = -0.5 / (bp.w[k] * bp.w[k]);
        sa[k] = bp.a[k];
    }
    __syncthreads();
    const uint32_t N = (uint32_t)n << ln;
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < N; e += gridDim.x * 256u) {
        const double x = ((e & (uint32_t)(n - 1)) + 1) * h, y = ((e >> ln) + 1) * h;
        double v = 0.0;
        for (int k = 0; k < K; ++k) {
            const double dx = x - scx[k], dy = y - scy[k];
            v = fma(sa[k], exp(sc[k] * fma(dx, dx, dy * dy)), v);
        }
        f[e] = v;
    }
}

// partial sums over a slice of the grid for bump k = blockIdx.y:
// S0 = sum g e, S1 = sum g e dx, S2 = sum g e dy, S3 = sum g e r^2
__global__ __launch_bounds__(256) void k_bumps_grad_part(BumpParams bp, const double *__restrict__ g,
                                                         double *__restrict__ part, int n, int ln,
                                                         double h)
{
    const int k = blockIdx.y;
    const double cx = bp.cx[k], cy = bp.cy[k], c = -0.5 / (bp.w[k] * bp.w[k]);
    const uint32_t N = (uint32_t)n << ln;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < N; e += gridDim.x * 256u) {
        const double dx = ((e & (uint32_t)(n - 1)) + 1) * h - cx, dy = ((e >> ln) + 1) * h - cy;
        const double r2 = fma(dx, dx, dy * dy);
        const double ge = g[e] * exp(c * r2);
        s0 += ge;
        s1 = fma(ge, dx, s1);
        s2 = fma(ge, dy, s2);
        s3 = fma(ge, r2, s3);
    }
    __shared__ double red[4][4];
    double v[4] = {s0, s1, s2, s3};
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double t = v[q];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) red[wv][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        part[((size_t)k * 4 + q) * gridDim.x + blockIdx.x] =
            (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

// one block per bump: fixed-order sum of the partials, then the factors
__global__ __launch_bounds__(64) void k_bumps_grad_finish(BumpParams bp, const double *__restrict__ part,
                                                          int nblk, double *gcx, double *gcy,
                                                          double *gw, double *ga)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    double S[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double *pq = part + ((size_t)k * 4 + q) * nblk;
        double t = 0.0;
        for (int b = lane; b < nblk; b += 64) t += pq[b];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        S[q] = t;
    }
    if (lane == 0) {
        const double a = bp.a[k], w = bp.w[k], iw2 = 1.0 / (w * w);
        if (ga) ga[k] = S[0];
        if (gcx) gcx[k] = a * iw2 * S[1];
        if (gcy) gcy[k] = a * iw2 * S[2];
        if (gw) gw[k] = a * iw2 / w * S[3];
    }
}

static int bump_grid(fmm_plan *pl)
{
    const int64_t N = pl->n * pl->n;
    int64_t b = (N + 2047) / 2048;
    return (int)(b < 1 ? 1 : b > 4096 ? 4096 : b);
}

int bumps_eval(fmm_plan *pl, int K, const double *cx, const double *cy, const double *w,
               const double *a, double *f, hipStream_t s)
{
    if (K < 1 || K > kBumpMax) return fail(pl, FMM_ERR_ARG, "K must be in [1, 256]");
    const BumpParams bp{cx, cy, w, a};
    hipLaunchKernelGGL(k_bumps_eval, dim3(bump_grid(pl)), dim3(256), 0, s, bp, K, f, (int)pl->n,
                       pl->L + 3, pl->h);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

// the two launches of a gradient evaluation, partials in part
// (K * 4 * kBumpBlocks doubles, every one written before it is read)
static int bumps_grad_launch(fmm_plan *pl, int K, const BumpParams &bp, const double *g,
                             double *part, double *gcx, double *gcy, double *gw, double *ga,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_bumps_grad_part, dim3(kBumpBlocks, K), dim3(256), 0, s, bp, g, part,
                       (int)pl->n, pl->L + 3, pl->h);
    hipLaunchKernelGGL(k_bumps_grad_finish, dim3(K), dim3(64), 0, s, bp, part, kBumpBlocks, gcx,
                       gcy, gw, ga);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int bumps_grad(fmm_plan *pl, int K, const double *cx, const double *cy, const double *w,
               const double *a, const double *g, double *gcx, double *gcy, double *gw,
               double *ga, hipStream_t s)
{
    if (K < 1 || K > kBumpMax) return fail(pl, FMM_ERR_ARG, "K must be in [1, 256]");
    if (!pl->bump_part)
        FMM_HIP(pl, hipMalloc(&pl->bump_part, (size_t)kBumpMax * 4 * kBumpBlocks * sizeof(double)));
    return bumps_grad_launch(pl, K, BumpParams{cx, cy, w, a}, g, pl->bump_part, gcx, gcy, gw, ga, s);
}

// Device address of the static workspace on the current device, looked up
// once per device (at plan setup, with the plan's device current).
int bumps_scratch_init(fmm_plan *pl)
{
    int dev = 0;
    FMM_HIP(pl, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(pl, FMM_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *addr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !addr)
            return fail(pl, FMM_ERR_DEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[dev] = static_cast<double *>(addr);
    }
    pl->bump_scratch = g_scratch_addr[dev];
    return FMM_OK;
}

int bumps_grad_noalloc(fmm_plan *pl, int K, const double *cx, const double *cy, const double *w,
                       const double *a, const double *g, double *gcx, double *gcy, double *gw,
                       double *ga, hipStream_t s)
{
    if (K < 1 || K > kBumpMax)
        return fail(pl, FMM_ERR_ARG,
                    "K must be in [1, 256] (the static workspace holds the partials of 256 bumps)");
    if (!pl->bump_scratch) return fail(pl, FMM_ERR_DEVICE, "static workspace address unknown");
    if ((int64_t)K * 4 * kBumpBlocks > kScratchDoubles)
        return fail(pl, FMM_ERR_ARG, "request exceeds the static workspace");
    return bumps_grad_launch(pl, K, BumpParams{cx, cy, w, a}, g, pl->bump_scratch, gcx, gcy, gw, ga,
                             s);
}

}  // namespace fmmprec
