// FMM on a point cloud (Sec. 5 of arXiv:1308.3339): u_i = sum_{j != i} q_j
// G(x_i - x_j), G = -(1/2pi) log r, on a uniform quadtree over a given root
// square with L = ceil(log4(N/64)) levels.
//
// Setup (tree.hip) sorts the points into leaves in Morton order on the
// device and keeps the sorted coordinates there.  An application gathers the
// charges into that order, builds leaf multipoles, reuses the level-generic
// M2M, M2L and L2L kernels of the grid path (whose expansions are indexed by
// row-major cell), and finishes with one block per target leaf: the sources
// of the near leaves around it (3x3 with the list rule, the disk of a MAC
// theta) are staged through LDS in chunks of their concatenated leaf
// segments, four waves split the sources, and the local expansion is
// evaluated at each target.  Blocks walk the leaves in Morton order, and
// consecutive Morton ranges go to the same accelerator die (XCD), so the
// near leaves a die stages are mostly its own.  FMM_FP32 plans run that near
// field pairwise in FP32 (the paper's P2P of Secs. 5.3 and 7.1: a polynomial
// logarithm and Kahan-compensated sums); the far field stays FP64.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "fmm_internal.h"
#include "log2_poly.h"

namespace fmmprec {

// level-generic stages of the grid path (fmm_grid.hip)
int points_upward_rest(fmm_plan *pl, hipStream_t s);
int points_m2l_down(fmm_plan *pl, hipStream_t s);

__device__ __forceinline__ double2 pcmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Morton index of leaf (lx, ly) and back (x bits even, y bits odd)
__device__ __forceinline__ uint32_t spread2(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
__device__ __forceinline__ uint32_t compact2(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}
__device__ __forceinline__ int morton2(int lx, int ly) { return (int)(spread2(lx) | (spread2(ly) << 1)); }

// Leaf of block b when leaves are walked in Morton order: the launch's
// blocks are dealt round-robin to the eight dies, so block b takes leaf
// (b mod 8) * (nleaf / 8) + b / 8 and each die works through one contiguous
// Morton range (a compact square of the domain).
__device__ __forceinline__ int leaf_of_block(int b, int nleaf)
{
    return (nleaf >= 64) ? (b & 7) * (nleaf >> 3) + (b >> 3) : b;
}

// Near-field sources of a target leaf: the concatenation of the sorted
// segments of its near leaves (rows |b| <= K, columns |a| <= kx(|b|)), in a
// fixed order.  seg_s[c] is the first sorted position of candidate c and
// seg_p[c] its offset in the concatenation (empty segments allowed);
// seg_p[nc] is the total.
constexpr int kMaxNearLeaves = (2 * kMaxK + 1) * (2 * kMaxK + 1);

__device__ __forceinline__ int near_segments(const int *__restrict__ start, int lx, int ly, int nl,
                                             int K, int kxp, int *seg_s, int *seg_p)
{
    const int side = 2 * K + 1, nc = side * side;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int b = c / side - K, a = c % side - K;
        const int kb = ((kxp >> (4 * (b < 0 ? -b : b))) & 15) - 1;
        const int qx = lx + a, qy = ly + b;
        int s0 = 0, len = 0;
        if ((a < 0 ? -a : a) <= kb && qx >= 0 && qx < nl && qy >= 0 && qy < nl) {
            const int m = morton2(qx, qy);
            s0 = start[m];
            len = start[m + 1] - s0;
        }
        seg_s[c] = s0;
        seg_p[c] = len;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int c = 0; c < nc; ++c) {
            const int len = seg_p[c];
            seg_p[c] = run;
            run += len;
        }
        seg_p[nc] = run;
    }
    __syncthreads();
    return nc;
}

// sorted position of element e of the concatenation: the last candidate
// whose offset is <= e (an empty segment shares its offset with the next)
__device__ __forceinline__ int near_source(const int *seg_s, const int *seg_p, int nc, int e)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_p[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return seg_s[lo] + (e - seg_p[lo]);
}

__global__ void k_gather(const double *__restrict__ q, const int *__restrict__ perm,
                         double *__restrict__ qs, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) qs[i] = q[perm[i]];
}

__global__ void k_scatter(const double *__restrict__ us, const int *__restrict__ perm,
                          double *__restrict__ u, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) u[perm[i]] = us[i];
}

// leaf multipoles, one wave per leaf: each lane accumulates the scaled
// series of its points (M~_0 = sum q, M~_k = -sum q tau^k / k with
// tau = (z - centre)/w) and the wave sums the lanes.
template <int P>
__global__ __launch_bounds__(256) void k_p2m_points(const double *__restrict__ px,
                                                    const double *__restrict__ py,
                                                    const double *__restrict__ qs,
                                                    const int *__restrict__ start,
                                                    double2 *__restrict__ M, int nl, double x0,
                                                    double y0, double w)
{
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (m >= nl * nl) return;
    const int lx = (int)compact2(m), ly = (int)compact2((uint32_t)m >> 1);
    const int leaf = ly * nl + lx;
    const double cx = x0 + (lx + 0.5) * w, cy = y0 + (ly + 0.5) * w, iw = 1.0 / w;
    double2 acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int j = start[m] + lane; j < start[m + 1]; j += 64) {
        const double c = qs[j];
        const double2 tau = make_double2((px[j] - cx) * iw, (py[j] - cy) * iw);
        double2 pw = make_double2(1.0, 0.0);
        acc[0].x += c;
#pragma unroll
        for (int k = 1; k < P; ++k) {
            pw = pcmul(pw, tau);
            acc[k].x += c * pw.x;
            acc[k].y += c * pw.y;
        }
    }
    const int64_t ncell = (int64_t)nl * nl;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double ax = acc[k].x, ay = acc[k].y;
        for (int o = 32; o > 0; o >>= 1) {
            ax += __shfl_xor(ax, o);
            ay += __shfl_xor(ay, o);
        }
        if (lane == 0) {
            const double f = (k == 0) ? 1.0 : -1.0 / (double)k;
            M[k * ncell + leaf] = make_double2(f * ax, f * ay);
        }
    }
}

// Natural logarithm of a positive, finite FP64 x for the pairwise near field,
// from the series log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),
// s = (m - 1)/(m + 1), after x = 2^e m with m in [1/sqrt2, sqrt2):
//   |s| <= 3 - 2 sqrt2 = 0.1716, z = s^2 <= 0.0295, and the terms after
//   z^9 s / 19 sum to less than 3e-17 of the result, so ten terms do;
//   1/(m + 1) is a hardware reciprocal refined by two Newton steps and s is
//   corrected once by its residual, which keeps s within about an ulp;
//   e ln 2 enters through a two-part constant (ln 2 = kLn2Hi + kLn2Lo).
// About 30 VALU instructions against the general-purpose library logarithm's
// 75, at an error of a few ulp (the parity tests hold the near field within
// 1e-12 of the oracle's libm sums).
constexpr double kLn2Hi = 0.69314718055994530942;            // nearest double to ln 2
constexpr double kLn2Lo = 2.3190468138462995584e-17;         // ln 2 - kLn2Hi
// 1/19, 1/17, ..., 1/3, the series coefficients, as data: the kernel loads
// them into scalar registers once (as literals the compiler holds them in
// vector registers and copies one before each multiply-add of the series)
__device__ double kSeriesInv[9] = {1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0,
                                   1.0 / 9.0,  1.0 / 7.0,  1.0 / 5.0,  1.0 / 3.0};

__device__ __forceinline__ double log_pos(double x, const double (&cs)[9])
{
    int e;
    double m = frexp(x, &e);                 // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double a = m - 1.0, d = m + 1.0;   // m - 1 is exact
    double y = __builtin_amdgcn_rcp(d);
    y = fma(y, fma(-d, y, 1.0), y);
    y = fma(y, fma(-d, y, 1.0), y);
    double sv = a * y;
    sv = fma(fma(-sv, d, a), y, sv);
    const double z = sv * sv;
    double p = cs[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) p = fma(p, z, cs[i]);
    const double s2 = 2.0 * sv;
    const double lm = fma(s2 * z, p, s2);
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
}

// near field + local expansion at the targets of one leaf per block
constexpr int kChunk = 1024;

template <int P>
__global__ __launch_bounds__(256) void k_leaf_points(const double *__restrict__ px,
                                                     const double *__restrict__ py,
                                                     const double *__restrict__ qs,
                                                     const int *__restrict__ start,
                                                     const double2 *__restrict__ Lt, LevelInfo lv,
                                                     int L, int far, double *__restrict__ us,
                                                     double x0, double y0, double w, int K,
                                                     int kxp)
{
    __shared__ double sx[kChunk], sy[kChunk], sqv[kChunk];
    __shared__ double red[4][64];
    __shared__ int seg_s[kMaxNearLeaves], seg_p[kMaxNearLeaves + 1];
    const int nl = 1 << L;
    const int m = leaf_of_block(blockIdx.x, nl * nl);
    const int lx = (int)compact2(m), ly = (int)compact2((uint32_t)m >> 1);
    const int leaf = ly * nl + lx;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t0 = start[m], t1 = start[m + 1];
    double2 Lc[P];
    if (far) {
        const int64_t ncell = (int64_t)nl * nl;
        const double2 *Ll = Lt + lv.off[L];
#pragma unroll
        for (int k = 0; k < P; ++k) Lc[k] = Ll[k * ncell + leaf];
    }
    const double cx = x0 + (lx + 0.5) * w, cy = y0 + (ly + 0.5) * w, iw = 1.0 / w;
    const int nc = near_segments(start, lx, ly, nl, K, kxp, seg_s, seg_p);
    const int ns = seg_p[nc];
    // sources of the near leaves (the 3x3 block with the list rule, the disk
    // of radius K with a MAC theta) in chunks through LDS, staged once for all
    // target slices when they fit one chunk
    auto stage = [&](int cb, int cnt) {
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += 256) {
            const int j = near_source(seg_s, seg_p, nc, cb + e);
            sx[e] = px[j];
            sy[e] = py[j];
            sqv[e] = qs[j];
        }
        __syncthreads();
    };
    const bool once = ns <= kChunk;
    if (once && t1 > t0) stage(0, ns);
    double cs[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) cs[i] = kSeriesInv[i];
    // targets in slices of up to 64: a slice of r targets gives each target
    // g = 64 / r lanes (lane = tl g + sub), and lane sub of wave wv takes the
    // sources e = wv + 4 sub (mod 4 g), so that a short last slice keeps the
    // lanes busy; a full slice is one target per lane, the sources in quarters
    for (int tb = t0; tb < t1; tb += 64) {
        const int r = min(64, t1 - tb), g = 64 / r;
        const int tl = lane / g, sub = lane - tl * g;
        const bool tv = tl < r;
        const double tx = tv ? px[tb + tl] : 0.0, ty = tv ? py[tb + tl] : 0.0;
        double acc = 0.0;
        for (int cb = 0; cb < ns; cb += kChunk) {
            const int cnt = min(kChunk, ns - cb);
            if (!once) stage(cb, cnt);
            if (tv) {
                for (int e = wv + 4 * sub; e < cnt; e += 4 * g) {
                    const double dx = tx - sx[e], dy = ty - sy[e];
                    const double r2 = dx * dx + dy * dy;
                    if (r2 > 0.0) acc = fma(sqv[e], log_pos(r2, cs), acc);
                }
            }
        }
        // per target, the partial sums in a fixed order: waves outer, sub-lanes
        // inner (a full slice: ((w0 + w1) + w2) + w3); the pairs summed
        // q log r^2, so half of it is the sum of q log r
        __syncthreads();
        red[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && lane < r) {
            const int t = tb + lane;
            double sum = 0.0;
            for (int w = 0; w < 4; ++w)
                for (int sb = 0; sb < g; ++sb) sum += red[w][lane * g + sb];
            acc = 0.5 * sum;
            double farv = 0.0;
            if (far) {
                const double2 tau = make_double2((px[t] - cx) * iw, (py[t] - cy) * iw);
                double2 pk = make_double2(1.0, 0.0);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    farv = fma(Lc[k].x, pk.x, fma(-Lc[k].y, pk.y, farv));
                    pk = pcmul(pk, tau);
                }
            }
            us[t] = -(acc + farv) * kInv2Pi;
        }
    }
}

// log2(x) for a normal FP32 x > 0: the exponent from the bits, the mantissa
// folded into [1/sqrt(2), sqrt(2)) and log2(m) = u p(u), u = m - 1 (Sec. 5.3's
// polynomial fit of log2(x)/(x - 1); coefficients in log2_poly.h).
__device__ __forceinline__ float log2_poly(float x)
{
    const uint32_t b = __float_as_uint(x);
    int e = (int)(b >> 23) - 127;
    float m = __uint_as_float((b & 0x007fffffu) | 0x3f800000u);
    if (m > 1.41421356f) {
        m *= 0.5f;
        ++e;
    }
    const float u = m - 1.0f;
    float p = kLog2Poly[kLog2PolyDegree];
#pragma unroll
    for (int i = kLog2PolyDegree - 1; i >= 0; --i) p = fmaf(p, u, kLog2Poly[i]);
    return fmaf(u, p, (float)e);
}

// FMM_FP32 form of k_leaf_points: the same blocks, waves and source chunks,
// with the pair sums in FP32 (Sec. 7.1).  Coordinates enter as FP32 offsets
// from the target leaf's centre (at most 1.5 leaf widths for the 3x3 near
// set), the charges as FP32; each lane sums q_j log2(r^2) over its quarter of
// the sources with Kahan compensation, and the four quarter sums, the factor
// ln2 / 2 and the FP64 local expansion are combined in FP64.  A pair with r^2
// below the smallest normal FP32 number (the target itself, or two points
// that FP32 offsets cannot tell apart) is left out like the self pair.
template <int P>
__global__ __launch_bounds__(256) void k_leaf_points_f32(const double *__restrict__ px,
                                                         const double *__restrict__ py,
                                                         const double *__restrict__ qs,
                                                         const int *__restrict__ start,
                                                         const double2 *__restrict__ Lt, LevelInfo lv,
                                                         int L, int far, double *__restrict__ us,
                                                         double x0, double y0, double w, int K,
                                                         int kxp)
{
    __shared__ float sx[kChunk], sy[kChunk], sqv[kChunk];
    __shared__ double red[4][64];
    __shared__ int seg_s[kMaxNearLeaves], seg_p[kMaxNearLeaves + 1];
    const int nl = 1 << L;
    const int m = leaf_of_block(blockIdx.x, nl * nl);
    const int lx = (int)compact2(m), ly = (int)compact2((uint32_t)m >> 1);
    const int leaf = ly * nl + lx;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t0 = start[m], t1 = start[m + 1];
    double2 Lc[P];
    if (far) {
        const int64_t ncell = (int64_t)nl * nl;
        const double2 *Ll = Lt + lv.off[L];
#pragma unroll
        for (int k = 0; k < P; ++k) Lc[k] = Ll[k * ncell + leaf];
    }
    const double cx = x0 + (lx + 0.5) * w, cy = y0 + (ly + 0.5) * w, iw = 1.0 / w;
    const int nc = near_segments(start, lx, ly, nl, K, kxp, seg_s, seg_p);
    const int ns = seg_p[nc];
    // sources staged and targets sliced as in k_leaf_points
    auto stage = [&](int cb, int cnt) {
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += 256) {
            const int j = near_source(seg_s, seg_p, nc, cb + e);
            sx[e] = (float)(px[j] - cx);
            sy[e] = (float)(py[j] - cy);
            sqv[e] = (float)qs[j];
        }
        __syncthreads();
    };
    const bool once = ns <= kChunk;
    if (once && t1 > t0) stage(0, ns);
    for (int tb = t0; tb < t1; tb += 64) {
        const int r = min(64, t1 - tb), g = 64 / r;
        const int tl = lane / g, sub = lane - tl * g;
        const bool tv = tl < r;
        const double tx = tv ? px[tb + tl] : 0.0, ty = tv ? py[tb + tl] : 0.0;
        const float txf = (float)(tx - cx), tyf = (float)(ty - cy);
        float ks = 0.0f, kc = 0.0f;   // Kahan sum of q log2(r^2) and its compensation
        for (int cb = 0; cb < ns; cb += kChunk) {
            const int cnt = min(kChunk, ns - cb);
            if (!once) stage(cb, cnt);
            if (tv) {
                for (int e = wv + 4 * sub; e < cnt; e += 4 * g) {
                    const float dx = txf - sx[e], dy = tyf - sy[e];
                    const float r2 = fmaf(dx, dx, dy * dy);
                    if (r2 >= FLT_MIN) {
                        const float y = fmaf(sqv[e], log2_poly(r2), -kc);
                        const float tsum = ks + y;
                        kc = (tsum - ks) - y;
                        ks = tsum;
                    }
                }
            }
        }
        __syncthreads();
        red[wv][lane] = ((double)ks - (double)kc) * (0.5 * kLn2);
        __syncthreads();
        if (wv == 0 && lane < r) {
            const int t = tb + lane;
            double acc = 0.0;
            for (int w = 0; w < 4; ++w)
                for (int sb = 0; sb < g; ++sb) acc += red[w][lane * g + sb];
            double farv = 0.0;
            if (far) {
                const double2 tau = make_double2((px[t] - cx) * iw, (py[t] - cy) * iw);
                double2 pk = make_double2(1.0, 0.0);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    farv = fma(Lc[k].x, pk.x, fma(-Lc[k].y, pk.y, farv));
                    pk = pcmul(pk, tau);
                }
            }
            us[t] = -(acc + farv) * kInv2Pi;
        }
    }
}

template <int P>
static int points_fmm_p(fmm_plan *pl, const double *q, double *u, hipStream_t s)
{
    const int N = (int)pl->n, nl = pl->nl, L = pl->L;
    const double w = pl->side / nl;
    const bool far = L >= 2;
    hipLaunchKernelGGL(k_gather, dim3((N + 255) / 256), dim3(256), 0, s, q, pl->perm, pl->qs, N);
    if (far) {
        {
            StageTimer t(pl, FMM_STAGE_P2M, s);
            hipLaunchKernelGGL(k_p2m_points<P>, dim3((nl * nl + 3) / 4), dim3(256), 0, s, pl->px,
                               pl->py, pl->qs, pl->leaf_start, pl->ws.M + pl->lv.off[L], nl,
                               pl->x0, pl->y0, w);
        }
        int st = points_upward_rest(pl, s);
        if (st != FMM_OK) return st;
        st = points_m2l_down(pl, s);
        if (st != FMM_OK) return st;
    }
    {
        StageTimer t(pl, FMM_STAGE_LEAF, s);
        if (pl->prec == FMM_FP32)
            hipLaunchKernelGGL(k_leaf_points_f32<P>, dim3(nl * nl), dim3(256), 0, s, pl->px, pl->py,
                               pl->qs, pl->leaf_start, pl->ws.Lt, pl->lv, L, far ? 1 : 0, pl->us,
                               pl->x0, pl->y0, w, pl->K, near_kx_packed(pl));
        else
            hipLaunchKernelGGL(k_leaf_points<P>, dim3(nl * nl), dim3(256), 0, s, pl->px, pl->py,
                               pl->qs, pl->leaf_start, pl->ws.Lt, pl->lv, L, far ? 1 : 0, pl->us,
                               pl->x0, pl->y0, w, pl->K, near_kx_packed(pl));
    }
    hipLaunchKernelGGL(k_scatter, dim3((N + 255) / 256), dim3(256), 0, s, pl->us, pl->perm, u, N);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int points_fmm(fmm_plan *pl, const double *q, double *u, hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, points_fmm_p, pl, q, u, s);
}

}  // namespace fmmprec
