// Tree construction for point-cloud plans on the device (Sec. 5.1, building
// the tree before the FMM passes; here the uniform quadtree of the plan):
//
//   1. keys       one thread per point: the leaf (lx, ly) by the clamp rule
//                 min(max(floor((x - x0)/side * 2^L), 0), 2^L - 1) and its
//                 Morton index (x bits in the even positions, y bits in the
//                 odd ones); the leaf histogram by integer atomics (exact).
//   2. leaf starts  exclusive scan of the histogram: leaf_start[m] is the
//                 first sorted position of Morton leaf m, leaf_start[4^L] = N.
//   3. order      stable least-significant-digit radix sort of (key, index)
//                 pairs, 8 bits per pass (ceil(2L / 8) passes): per-block
//                 digit counts, an exclusive scan over (digit, block) in
//                 digit-major order, and a scatter that ranks equal digits
//                 by round, wave and lane, so that each pass keeps the order
//                 of the one before it.  Points of one leaf therefore keep
//                 their original order.
//
// The scans are plain two-level block scans (1024 elements per block)
// applied recursively to the block sums.
#include <algorithm>
#include <utility>

#include "fmm_internal.h"

namespace fmmprec {

constexpr int kScanBlock = 1024;       // elements per scan block (256 threads x 4)
constexpr int kSortItems = 2048;       // items per radix block (256 threads x 8 rounds)
constexpr int kSortRounds = kSortItems / 256;

__host__ __device__ __forceinline__ uint32_t spread_bits(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// leaf keys and histogram; bad[0] is set when a coordinate is not finite
__global__ __launch_bounds__(256) void k_point_keys(const double *__restrict__ x,
                                                    const double *__restrict__ y, int N,
                                                    double x0, double y0, double side, int nl,
                                                    uint32_t *__restrict__ key,
                                                    int *__restrict__ idx,
                                                    int *__restrict__ hist, int *__restrict__ bad)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double xi = x[i], yi = y[i];
    uint32_t k = 0;
    if (!isfinite(xi) || !isfinite(yi)) {
        atomicOr(bad, 1);
    } else {
        double fx = floor((xi - x0) / side * nl), fy = floor((yi - y0) / side * nl);
        fx = fmin(fmax(fx, 0.0), (double)(nl - 1));
        fy = fmin(fmax(fy, 0.0), (double)(nl - 1));
        k = spread_bits((uint32_t)fx) | (spread_bits((uint32_t)fy) << 1);
    }
    key[i] = k;
    idx[i] = i;
    atomicAdd(&hist[k], 1);
}

// exclusive scan of blocks of kScanBlock ints (in may equal out); the block
// totals go to sums (when not null)
__global__ __launch_bounds__(256) void k_scan_block(const int *in, int *out, int64_t M, int *sums)
{
    __shared__ int wtot[4];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
    int v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = base + i < M ? in[base + i] : 0;
    const int t = v[0] + v[1] + v[2] + v[3];
    // inclusive scan of the thread totals within the wave
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int s = t;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(s, o);
        if (lane >= o) s += u;
    }
    if (lane == 63) wtot[wv] = s;
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wv; ++w) woff += wtot[w];
    int run = woff + s - t;   // exclusive prefix of this thread's first element
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = v[i];
        if (base + i < M) out[base + i] = run;
        run += e;
    }
    if (sums && threadIdx.x == 255) sums[blockIdx.x] = woff + s;
}

__global__ __launch_bounds__(256) void k_scan_add(int *out, int64_t M, const int *offs)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
    const int a = offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < M) out[base + i] += a;
}

// exclusive scan of M ints in place; tmp holds at least scan_tmp_ints(M)
static int64_t scan_tmp_ints(int64_t M)
{
    int64_t t = 0;
    while (M > kScanBlock) {
        M = (M + kScanBlock - 1) / kScanBlock;
        t += M;
    }
    return t + 1;
}

static void scan_exclusive(int *a, int64_t M, int *tmp, hipStream_t s)
{
    const int64_t nb = (M + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(256), 0, s, a, a, M, (int *)nullptr);
        return;
    }
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(256), 0, s, a, a, M, tmp);
    scan_exclusive(tmp, nb, tmp + nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, a, M, tmp);
}

// per-block counts of one 8-bit digit, stored digit-major: cnt[d * nblk + b]
__global__ __launch_bounds__(256) void k_radix_count(const uint32_t *__restrict__ key, int N,
                                                     int shift, int *__restrict__ cnt, int nblk)
{
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortItems;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < N) atomicAdd(&h[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// stable scatter of one pass: the item at position i of block b goes to
// offs[d * nblk + b] + (earlier items of this block with digit d), where
// "earlier" is round-major, then wave, then lane: the input order.
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                       const int *__restrict__ iin,
                                                       uint32_t *__restrict__ kout,
                                                       int *__restrict__ iout, int N, int shift,
                                                       const int *__restrict__ offs, int nblk)
{
    __shared__ int run[256];
    __shared__ int wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    run[tid] = 0;
    const int64_t base = (int64_t)blockIdx.x * kSortItems;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * 256 + tid;
        const bool valid = i < N;
        const uint32_t k = valid ? kin[i] : 0u;
        const int ix = valid ? iin[i] : 0;
        const uint32_t d = (k >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        __syncthreads();
        if (valid && rank == 0) wcnt[wv][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = offs[(int64_t)d * nblk + blockIdx.x] + run[d] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
            kout[pos] = k;
            iout[pos] = ix;
        }
        __syncthreads();
        run[tid] += (wcnt[0][tid] + wcnt[1][tid]) + (wcnt[2][tid] + wcnt[3][tid]);
        __syncthreads();
    }
}

__global__ void k_gather_xy(const double *__restrict__ x, const double *__restrict__ y,
                            const int *__restrict__ perm, double *__restrict__ px,
                            double *__restrict__ py, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) {
        const int j = perm[i];
        px[i] = x[j];
        py[i] = y[j];
    }
}

// Builds pl->perm, pl->leaf_start, pl->px, pl->py from the caller's device
// coordinates.  Temporary buffers are freed before it returns.
int points_setup(fmm_plan *pl, const double *dx, const double *dy, hipStream_t s)
{
    const int64_t N64 = pl->n;
    if (N64 > (int64_t)1 << 30) return fail(pl, FMM_ERR_ARG, "POINTS n must be <= 2^30");
    const int N = (int)N64, L = pl->L, nl = pl->nl;
    const int64_t nleaf = (int64_t)nl * nl;
    const int nblk = (N + kSortItems - 1) / kSortItems;
    const int passes = (2 * L + 7) / 8;
    const int64_t M = (int64_t)256 * nblk;
    const int64_t tmp_ints = std::max(scan_tmp_ints(nleaf + 1), scan_tmp_ints(M));
    FMM_HIP(pl, hipMalloc(&pl->perm, N64 * sizeof(int)));
    FMM_HIP(pl, hipMalloc(&pl->leaf_start, (nleaf + 1) * sizeof(int)));
    FMM_HIP(pl, hipMalloc(&pl->px, N64 * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->py, N64 * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->qs, N64 * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->us, N64 * sizeof(double)));
    // scratch of the build: keys (two), indices (one more), digit counts, scan, flag
    uint32_t *k0 = nullptr, *k1 = nullptr;
    int *i1 = nullptr, *cnt = nullptr, *tmp = nullptr, *bad = nullptr;
    auto release = [&]() {
        for (void *ptr : {(void *)k0, (void *)k1, (void *)i1, (void *)cnt, (void *)tmp, (void *)bad})
            if (ptr) (void)hipFree(ptr);
    };
    if (hipMalloc(&k0, N64 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&k1, N64 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&i1, N64 * sizeof(int)) != hipSuccess ||
        hipMalloc(&cnt, M * sizeof(int)) != hipSuccess ||
        hipMalloc(&tmp, tmp_ints * sizeof(int)) != hipSuccess || hipMalloc(&bad, sizeof(int)) != hipSuccess) {
        release();
        return fail(pl, FMM_ERR_ALLOC, "tree construction scratch allocation failed");
    }
    int *hist = pl->leaf_start;
    int *i0 = pl->perm;
    hipError_t e = hipMemsetAsync(hist, 0, (nleaf + 1) * sizeof(int), s);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), s);
    if (e != hipSuccess) {
        release();
        return fail(pl, FMM_ERR_DEVICE, std::string("tree setup: ") + hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_point_keys, dim3((N + 255) / 256), dim3(256), 0, s, dx, dy, N, pl->x0,
                       pl->y0, pl->side, nl, k0, i0, hist, bad);
    scan_exclusive(hist, nleaf + 1, tmp, s);
    // radix passes ping-pong between (k0, i0) and (k1, i1); an odd count ends in (k1, i1)
    uint32_t *ka = k0, *kb = k1;
    int *ia = i0, *ib = i1;
    for (int pass = 0; pass < passes; ++pass) {
        hipLaunchKernelGGL(k_radix_count, dim3(nblk), dim3(256), 0, s, ka, N, 8 * pass, cnt, nblk);
        scan_exclusive(cnt, M, tmp, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(256), 0, s, ka, ia, kb, ib, N, 8 * pass,
                           cnt, nblk);
        std::swap(ka, kb);
        std::swap(ia, ib);
    }
    if (ia != pl->perm) e = hipMemcpyAsync(pl->perm, ia, N64 * sizeof(int), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gather_xy, dim3((N + 255) / 256), dim3(256), 0, s, dx, dy, pl->perm,
                           pl->px, pl->py, N);
        e = hipGetLastError();
    }
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) return fail(pl, FMM_ERR_DEVICE, std::string("tree setup: ") + hipGetErrorString(e));
    if (hbad) return fail(pl, FMM_ERR_ARG, "POINTS coordinates must be finite");
    return FMM_OK;
}

}  // namespace fmmprec
