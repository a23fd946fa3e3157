// FMM on a point cloud (Sec. 5 of arXiv:1308.3339): u_i = sum_{j != i} q_j
// G(x_i - x_j), G = -(1/2pi) log r, on a uniform quadtree over a given root
// square with L = ceil(log4(N/64)) levels.
//
// Setup bins the points into leaves (stable counting sort by leaf, leaves in
// row-major order) and keeps the sorted coordinates on the device.  An
// application gathers the charges into leaf order, builds leaf multipoles,
// reuses the level-generic M2M, M2L and L2L kernels of the grid path, and
// finishes with one block per target leaf: the sources of the near leaves
// around it (3x3 with the list rule, the disk of a MAC theta) are staged
// through LDS in chunks, four waves split the sources, and the local
// expansion is evaluated at each target.  FMM_FP32 plans run that near
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
    const int leaf = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (leaf >= nl * nl) return;
    const int lx = leaf % nl, ly = leaf / nl;
    const double cx = x0 + (lx + 0.5) * w, cy = y0 + (ly + 0.5) * w, iw = 1.0 / w;
    double2 acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int j = start[leaf] + lane; j < start[leaf + 1]; j += 64) {
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
    __shared__ double red[3][64];
    const int nl = 1 << L;
    const int leaf = blockIdx.x;
    const int lx = leaf % nl, ly = leaf / nl;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t0 = start[leaf], t1 = start[leaf + 1];
    double2 Lc[P];
    if (far) {
        const int64_t ncell = (int64_t)nl * nl;
        const double2 *Ll = Lt + lv.off[L];
#pragma unroll
        for (int k = 0; k < P; ++k) Lc[k] = Ll[k * ncell + leaf];
    }
    const double cx = x0 + (lx + 0.5) * w, cy = y0 + (ly + 0.5) * w, iw = 1.0 / w;
    // targets in slices of 64; sources of the near leaves (the 3x3 block with
    // the list rule, the disk of radius K with a MAC theta) in chunks through LDS
    for (int tb = t0; tb < t1; tb += 64) {
        const int t = tb + lane;
        const bool tv = t < t1;
        const double tx = tv ? px[t] : 0.0, ty = tv ? py[t] : 0.0;
        double acc = 0.0;
        for (int b = -K; b <= K; ++b) {
            const int qy = ly + b, kb = ((kxp >> (4 * (b < 0 ? -b : b))) & 15) - 1;
            if (qy < 0 || qy >= nl || kb < 0) continue;
            const int qx0 = max(lx - kb, 0), qx1 = min(lx + kb, nl - 1);
            // the leaves of one row of the near set are contiguous in the sorted order
            const int s0 = start[qy * nl + qx0], s1 = start[qy * nl + qx1 + 1];
            for (int cb = s0; cb < s1; cb += kChunk) {
                const int cnt = min(kChunk, s1 - cb);
                __syncthreads();
                for (int e = threadIdx.x; e < cnt; e += 256) {
                    sx[e] = px[cb + e];
                    sy[e] = py[cb + e];
                    sqv[e] = qs[cb + e];
                }
                __syncthreads();
                if (tv) {
                    for (int e = wv; e < cnt; e += 4) {
                        const double dx = tx - sx[e], dy = ty - sy[e];
                        const double r2 = dx * dx + dy * dy;
                        if (r2 > 0.0) acc = fma(sqv[e], log(sqrt(r2)), acc);
                    }
                }
            }
        }
        // sum the four source quarters: ((w0 + w1) + w2) + w3
        __syncthreads();
        if (wv > 0) red[wv - 1][lane] = acc;
        __syncthreads();
        if (wv == 0 && tv) {
            acc = ((acc + red[0][lane]) + red[1][lane]) + red[2][lane];
            double farv = 0.0;
            if (far) {
                const double2 tau = make_double2((tx - cx) * iw, (ty - cy) * iw);
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
    __shared__ double red[3][64];
    const int nl = 1 << L;
    const int leaf = blockIdx.x;
    const int lx = leaf % nl, ly = leaf / nl;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t0 = start[leaf], t1 = start[leaf + 1];
    double2 Lc[P];
    if (far) {
        const int64_t ncell = (int64_t)nl * nl;
        const double2 *Ll = Lt + lv.off[L];
#pragma unroll
        for (int k = 0; k < P; ++k) Lc[k] = Ll[k * ncell + leaf];
    }
    const double cx = x0 + (lx + 0.5) * w, cy = y0 + (ly + 0.5) * w, iw = 1.0 / w;
    for (int tb = t0; tb < t1; tb += 64) {
        const int t = tb + lane;
        const bool tv = t < t1;
        const double tx = tv ? px[t] : 0.0, ty = tv ? py[t] : 0.0;
        const float txf = (float)(tx - cx), tyf = (float)(ty - cy);
        float ks = 0.0f, kc = 0.0f;   // Kahan sum of q log2(r^2) and its compensation
        for (int b = -K; b <= K; ++b) {
            const int qy = ly + b, kb = ((kxp >> (4 * (b < 0 ? -b : b))) & 15) - 1;
            if (qy < 0 || qy >= nl || kb < 0) continue;
            const int qx0 = max(lx - kb, 0), qx1 = min(lx + kb, nl - 1);
            const int s0 = start[qy * nl + qx0], s1 = start[qy * nl + qx1 + 1];
            for (int cb = s0; cb < s1; cb += kChunk) {
                const int cnt = min(kChunk, s1 - cb);
                __syncthreads();
                for (int e = threadIdx.x; e < cnt; e += 256) {
                    sx[e] = (float)(px[cb + e] - cx);
                    sy[e] = (float)(py[cb + e] - cy);
                    sqv[e] = (float)qs[cb + e];
                }
                __syncthreads();
                if (tv) {
                    for (int e = wv; e < cnt; e += 4) {
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
        }
        double acc = ((double)ks - (double)kc) * (0.5 * kLn2);
        __syncthreads();
        if (wv > 0) red[wv - 1][lane] = acc;
        __syncthreads();
        if (wv == 0 && tv) {
            acc = ((acc + red[0][lane]) + red[1][lane]) + red[2][lane];
            double farv = 0.0;
            if (far) {
                const double2 tau = make_double2((tx - cx) * iw, (ty - cy) * iw);
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

int points_setup(fmm_plan *pl, const double *dx, const double *dy, hipStream_t s)
{
    const int64_t N = pl->n;
    if (N > (int64_t)1 << 30) return fail(pl, FMM_ERR_ARG, "POINTS n must be <= 2^30");
    std::vector<double> hx(N), hy(N);
    FMM_HIP(pl, hipMemcpyAsync(hx.data(), dx, N * sizeof(double), hipMemcpyDeviceToHost, s));
    FMM_HIP(pl, hipMemcpyAsync(hy.data(), dy, N * sizeof(double), hipMemcpyDeviceToHost, s));
    FMM_HIP(pl, hipStreamSynchronize(s));
    const int nl = pl->nl;
    const int64_t nleaf = (int64_t)nl * nl;
    std::vector<int> leaf(N), start(nleaf + 1, 0), perm(N);
    for (int64_t i = 0; i < N; ++i) {
        if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]))
            return fail(pl, FMM_ERR_ARG, "POINTS coordinates must be finite");
        double fx = std::floor((hx[i] - pl->x0) / pl->side * nl);
        double fy = std::floor((hy[i] - pl->y0) / pl->side * nl);
        fx = std::min(std::max(fx, 0.0), (double)(nl - 1));
        fy = std::min(std::max(fy, 0.0), (double)(nl - 1));
        leaf[i] = (int)fy * nl + (int)fx;
        start[leaf[i] + 1]++;
    }
    for (int64_t c = 0; c < nleaf; ++c) start[c + 1] += start[c];
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < N; ++i) perm[fill[leaf[i]]++] = (int)i;   // stable: ties by index
    std::vector<double> sx(N), sy(N);
    for (int64_t i = 0; i < N; ++i) {
        sx[i] = hx[perm[i]];
        sy[i] = hy[perm[i]];
    }
    FMM_HIP(pl, hipMalloc(&pl->perm, N * sizeof(int)));
    FMM_HIP(pl, hipMalloc(&pl->leaf_start, (nleaf + 1) * sizeof(int)));
    FMM_HIP(pl, hipMalloc(&pl->px, N * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->py, N * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->qs, N * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->us, N * sizeof(double)));
    FMM_HIP(pl, hipMemcpy(pl->perm, perm.data(), N * sizeof(int), hipMemcpyHostToDevice));
    FMM_HIP(pl, hipMemcpy(pl->leaf_start, start.data(), (nleaf + 1) * sizeof(int), hipMemcpyHostToDevice));
    FMM_HIP(pl, hipMemcpy(pl->px, sx.data(), N * sizeof(double), hipMemcpyHostToDevice));
    FMM_HIP(pl, hipMemcpy(pl->py, sy.data(), N * sizeof(double), hipMemcpyHostToDevice));
    return FMM_OK;
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
