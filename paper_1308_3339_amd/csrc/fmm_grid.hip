// FMM stages for grid plans on gfx950 (Sec. 5 of arXiv:1308.3339).
//
// The grid is uniform, so every leaf holds the same 8 x 8 point pattern and
// every translation operator depends only on a small integer offset.  The
// stages are:
//   P2M    (Sec. 5.3 item 1)  leaf multipoles, a fixed p x 64 weight table
//   M2M    (item 2)           4 fixed quadrant matrices, one launch per level
//   M2L    (item 3)           one launch for all levels; a block is a 16x16
//                             tile of target cells and a third of their
//                             27-entry lists, sources staged in LDS
//   L2L    (item 4)           Taylor shift by the child offset, per level
//   L2P + P2P (item 5, Sec. 5.1)  one fused leaf kernel; the near field is a
//                             3x3-leaf restricted convolution whose kernel
//                             values log(h|d|) are wave-uniform (scalar
//                             registers) because lanes map to leaves
//
// Expansions are scaled by the cell width w of their level (M~_k = M_k/w^k,
// L~_k = L_k w^k), which makes M2M, M2L and L2L level independent.
#include "fmm_internal.h"

namespace fmmprec {

__device__ __forceinline__ void cmac(double2 &acc, double2 a, double2 b)
{
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// P2M on grid leaves: M~_k = qscale * sum_j W[k][j] q_j with
// W[0][j] = 1, W[k][j] = -tau_j^k / k, tau_j = ((a-3.5) + i(b-3.5)) / 8.
// Block: 256 threads = 32 leaves of one leaf row x 8 coefficient lanes.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_p2m_grid(const double *__restrict__ q, double qscale,
                                                  const double2 *__restrict__ W,
                                                  double2 *__restrict__ M, int n, int nl)
{
    __shared__ double sq[8][256 + 2];
    __shared__ double2 sw[P][64];
    const int tid = threadIdx.x;
    const int ly = blockIdx.y;
    const int lx0 = blockIdx.x * 32;
    for (int e = tid; e < P * 64; e += 256) sw[e >> 6][e & 63] = W[e];
    const int gx = lx0 * 8 + tid;
    for (int b = 0; b < 8; ++b)
        sq[b][tid] = (gx < n) ? q[(size_t)(ly * 8 + b) * n + gx] : 0.0;
    __syncthreads();
    const int lxl = tid >> 3, g = tid & 7;
    const int lx = lx0 + lxl;
    if (lx >= nl) return;
    const int64_t ncell = (int64_t)nl * nl;
    const int64_t cell = (int64_t)ly * nl + lx;
    for (int k = g; k < P; k += 8) {
        double ax = 0.0, ay = 0.0;
#pragma unroll 8
        for (int j = 0; j < 64; ++j) {
            const double v = sq[j >> 3][lxl * 8 + (j & 7)];
            ax = fma(sw[k][j].x, v, ax);
            ay = fma(sw[k][j].y, v, ay);
        }
        M[k * ncell + cell] = make_double2(ax * qscale, ay * qscale);
    }
}

// ---------------------------------------------------------------------------
// M2M: parent (ix, iy) of level l from its 4 children at level l+1.
// A[qd][n][k] (k <= n), qd = 2*(child y parity) + (child x parity).
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_m2m(const double2 *__restrict__ Mc,
                                             double2 *__restrict__ Mp,
                                             const double2 *__restrict__ A, int ncp)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= ncp * ncp) return;
    const int ix = idx % ncp, iy = idx / ncp;
    const int ncc = 2 * ncp;
    const int64_t nC = (int64_t)ncc * ncc, nP = (int64_t)ncp * ncp;
    double2 acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = make_double2(0.0, 0.0);
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
        const int cx = 2 * ix + (qd & 1), cy = 2 * iy + (qd >> 1);
        const int64_t cc = (int64_t)cy * ncc + cx;
        double2 mc[P];
#pragma unroll
        for (int k = 0; k < P; ++k) mc[k] = Mc[k * nC + cc];
        const double2 *Aq = A + qd * P * P;
#pragma unroll
        for (int nn = 0; nn < P; ++nn)
#pragma unroll
            for (int k = 0; k <= nn; ++k) cmac(acc[nn], Aq[nn * P + k], mc[k]);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) Mp[k * nP + idx] = acc[k];
}

// ---------------------------------------------------------------------------
// M2L for all levels 2..L in one launch.
// Scaled Hankel form of Sec. 5.3 item 3: with d^ = offset in cell widths,
//   L~_n = a_n sum_k H_{n+k} M'_k,  a_n = (-1)^n/n!,
//   M'_0 = -M~_0, M'_k = M~_k/(k-1)!,
//   H_0 = -(log|d^| + log w), H_m = (m-1)!/d^^m.
// A block is a 16x16 tile of target cells (the whole level if it is
// smaller) and one of the three 9-entry thirds of their interaction lists.
// Wave w serves the cells of parity class (w&1, w>>1): those share one list
// shape, so the offset and its Hankel generators are wave-uniform.
// Sources (20x20 cells around the tile) are staged in LDS split by parity,
// which makes the per-offset LDS reads of a wave consecutive.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_m2l(const M2LItem *__restrict__ items,
                                             const double2 *__restrict__ M,
                                             double2 *__restrict__ Lp0,
                                             double2 *__restrict__ Lp1,
                                             double2 *__restrict__ Lp2, LevelInfo lv,
                                             const double2 *__restrict__ hank,
                                             const int4 *__restrict__ offs,
                                             const double *__restrict__ a_n,
                                             const double *__restrict__ b_k)
{
    extern __shared__ double2 sm[];  // [P][RW*RW], parity split
    const M2LItem it = items[blockIdx.x];
    const int l = it.level, nc = 1 << l;
    const int tw = nc < 16 ? nc : 16;
    const int RW = tw + 4, RH = RW >> 1, SUB = RH * RH, RR = RW * RW;
    const int64_t ncell = (int64_t)nc * nc;
    const double2 *Ml = M + lv.off[l];
    for (int e = threadIdx.x; e < P * RR; e += 256) {
        const int k = e / RR, r = e - k * RR;
        const int sy = r / RW, sx = r - sy * RW;
        const int gx = it.tx0 - 2 + sx, gy = it.ty0 - 2 + sy;
        double2 v = make_double2(0.0, 0.0);
        if (gx >= 0 && gx < nc && gy >= 0 && gy < nc) {
            v = Ml[k * ncell + (int64_t)gy * nc + gx];
            const double bk = b_k[k];
            v.x *= bk;
            v.y *= bk;
        }
        sm[k * RR + ((sy & 1) * 2 + (sx & 1)) * SUB + (sy >> 1) * RH + (sx >> 1)] = v;
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int px = wave & 1, py = wave >> 1;
    const int ltx = 2 * (lane & 7) + px, lty = 2 * (lane >> 3) + py;
    const bool active = ltx < tw && lty < tw;
    double2 acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = make_double2(0.0, 0.0);
    const double logw = lv.logw[l];
    const int4 *ol = offs + wave * 27 + it.group * 9;
    if (active) {
        for (int o = 0; o < 9; ++o) {
            const int4 od = ol[o];
            const double2 *H = hank + od.z * (2 * P - 1);
            const int sx = ltx + od.x + 2, sy = lty + od.y + 2;
            const int sidx = ((sy & 1) * 2 + (sx & 1)) * SUB + (sy >> 1) * RH + (sx >> 1);
            double2 m[P];
#pragma unroll
            for (int k = 0; k < P; ++k) m[k] = sm[k * RR + sidx];
            // anti-diagonal order: each generator H_s is used by all (n, k), n+k = s
#pragma unroll
            for (int s = 0; s < 2 * P - 1; ++s) {
                double2 h = H[s];
                if (s == 0) h.x -= logw;
#pragma unroll
                for (int nn = (s < P ? 0 : s - P + 1); nn <= (s < P ? s : P - 1); ++nn)
                    cmac(acc[nn], h, m[s - nn]);
            }
        }
    }
    if (!active) return;
    const int tx = it.tx0 + ltx, ty = it.ty0 + lty;
    double2 *out = (it.group == 0 ? Lp0 : (it.group == 1 ? Lp1 : Lp2)) + lv.off[l];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double an = a_n[k];
        out[k * ncell + (int64_t)ty * nc + tx] = make_double2(an * acc[k].x, an * acc[k].y);
    }
}

// Taylor shift of a local expansion to a child: L~child_n = 2^-n sum_{k>=n}
// C(k,n) c^(k-n) L~parent_k with c = (child centre - parent centre)/w_parent
// = ((ex - 1/2) + i(ey - 1/2)) / 2.  Repeated synthetic division.
template <int P>
__device__ __forceinline__ void l2l_shift(double2 a[P], int ex, int ey)
{
    const double2 c = make_double2(0.5 * (ex - 0.5), 0.5 * (ey - 0.5));
#pragma unroll
    for (int i = 0; i < P - 1; ++i)
#pragma unroll
        for (int k = P - 2; k >= i; --k) cmac(a[k], c, a[k + 1]);
    double sc = 1.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        a[k].x *= sc;
        a[k].y *= sc;
        sc *= 0.5;
    }
}

// Local expansion of cell (ix, iy) at level l: sum of its M2L partials plus
// the shifted expansion of its parent (levels >= 3).
template <int P>
__device__ __forceinline__ void local_expansion(const double2 *__restrict__ Lp0,
                                                const double2 *__restrict__ Lp1,
                                                const double2 *__restrict__ Lp2,
                                                const double2 *__restrict__ Lt,
                                                const LevelInfo &lv, int l, int ix, int iy,
                                                double2 out[P])
{
    const int nc = 1 << l;
    const int64_t ncell = (int64_t)nc * nc, cell = (int64_t)iy * nc + ix;
    if (l >= 3) {
        const int ncp = nc >> 1;
        const int64_t nP = (int64_t)ncp * ncp, pc = (int64_t)(iy >> 1) * ncp + (ix >> 1);
        const double2 *Lpar = Lt + lv.off[l - 1];
#pragma unroll
        for (int k = 0; k < P; ++k) out[k] = Lpar[k * nP + pc];
        l2l_shift<P>(out, ix & 1, iy & 1);
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) out[k] = make_double2(0.0, 0.0);
    }
    const int64_t o = lv.off[l];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double2 a = Lp0[o + k * ncell + cell], b = Lp1[o + k * ncell + cell],
                      c = Lp2[o + k * ncell + cell];
        out[k].x += (a.x + b.x) + c.x;
        out[k].y += (a.y + b.y) + c.y;
    }
}

// L2L cascade: Lt[l] for one level (2 <= l <= L-1)
template <int P>
__global__ __launch_bounds__(256) void k_l2l(const double2 *__restrict__ Lp0,
                                             const double2 *__restrict__ Lp1,
                                             const double2 *__restrict__ Lp2,
                                             double2 *__restrict__ Lt, LevelInfo lv, int l)
{
    const int nc = 1 << l;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= nc * nc) return;
    double2 a[P];
    local_expansion<P>(Lp0, Lp1, Lp2, Lt, lv, l, idx % nc, idx / nc, a);
    const int64_t ncell = (int64_t)nc * nc;
#pragma unroll
    for (int k = 0; k < P; ++k) Lt[lv.off[l] + k * ncell + idx] = a[k];
}

// ---------------------------------------------------------------------------
// Fused leaf stage for grid plans:
//   u = -(1/2pi) [ qscale * sum_{3x3 leaves} q_j T(d_ij) + Re sum_k L~_k tau^k ]
// T(d) = log(h|d|) for lattice offsets d != 0 and log(eps h) for d = 0 (the
// regularised self term).  Block = 8x8 leaves; lane = leaf; wave w serves
// target rows 2w, 2w+1 of every leaf (16 targets per lane).  For a fixed
// source position all lanes need the same T values, so T rows are read with
// scalar loads and broadcast, and the q tile sits in LDS as [pos][leaf].
// ---------------------------------------------------------------------------
struct LeafArgs {
    const double *q;
    double qscale;
    double *u;
    const double2 *Lp0, *Lp1, *Lp2, *Lt;
    const double *ktab;   // [31][31]
    const double2 *l2p;   // [64][P]
    LevelInfo lv;
    int n, nl, L, far;
};

template <int P>
__global__ __launch_bounds__(256) void k_leaf_grid(LeafArgs a)
{
    __shared__ double sq[64 * 100];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, nl = a.nl;
    const int TX0 = blockIdx.x * 8, TY0 = blockIdx.y * 8;
    const int X0 = (TX0 - 1) * 8, Y0 = (TY0 - 1) * 8;
    for (int e = tid; e < 6400; e += 256) {
        const int yy = e / 80, xx = e - yy * 80;
        const int gx = X0 + xx, gy = Y0 + yy;
        double v = 0.0;
        if (gx >= 0 && gx < n && gy >= 0 && gy < n) v = a.q[(size_t)gy * n + gx];
        sq[((yy & 7) * 8 + (xx & 7)) * 100 + (yy >> 3) * 10 + (xx >> 3)] = v;
    }
    __syncthreads();
    const int lx = lane & 7, ly = lane >> 3;
    const int gLx = TX0 + lx, gLy = TY0 + ly;
    const bool active = gLx < nl && gLy < nl;
    const int ty0 = 2 * wave;
    const int cleaf = (ly + 1) * 10 + (lx + 1);
    double acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.0;
    const double *__restrict__ kt = a.ktab;
    for (int oy = -1; oy <= 1; ++oy) {
        for (int sy = 0; sy < 8; ++sy) {
            const int dy0 = 8 * oy + sy - ty0;  // row ty0 sees dy0, row ty0+1 sees dy0-1
            const double *T0 = kt + (dy0 + 15) * 31 + 8;
            const double *T1 = kt + (dy0 + 14) * 31 + 8;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                double w0[15], w1[15];
#pragma unroll
                for (int c = 0; c < 15; ++c) {
                    w0[c] = T0[8 * ox + c];
                    w1[c] = T1[8 * ox + c];
                }
                const int sl = cleaf + oy * 10 + ox;
#pragma unroll
                for (int sx = 0; sx < 8; ++sx) {
                    const double v = sq[(sy * 8 + sx) * 100 + sl];
#pragma unroll
                    for (int tx = 0; tx < 8; ++tx) {
                        acc[tx] = fma(w0[sx - tx + 7], v, acc[tx]);
                        acc[8 + tx] = fma(w1[sx - tx + 7], v, acc[8 + tx]);
                    }
                }
            }
        }
    }
    if (!active) return;
    double far[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) far[t] = 0.0;
    if (a.far) {
        double2 Lc[P];
        local_expansion<P>(a.Lp0, a.Lp1, a.Lp2, a.Lt, a.lv, a.L, gLx, gLy, Lc);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const double2 *tp = a.l2p + ((ty0 + (t >> 3)) * 8 + (t & 7)) * P;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) s = fma(Lc[k].x, tp[k].x, fma(-Lc[k].y, tp[k].y, s));
            far[t] = s;
        }
    }
    const double qs = a.qscale;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int gy = gLy * 8 + ty0 + (t >> 3), gx = gLx * 8 + (t & 7);
        a.u[(size_t)gy * n + gx] = -(fma(qs, acc[t], far[t])) * kInv2Pi;
    }
}

// Lattice coordinates (in units of h) of ring node t (counter-clockwise).
__device__ __forceinline__ void ring_node(int t, int n, int &Ix, int &Iy)
{
    const int s = t / n, k = t - s * n;
    if (s == 0) { Ix = k + 1; Iy = 0; }
    else if (s == 1) { Ix = n + 1; Iy = k + 1; }
    else if (s == 2) { Ix = n - k; Iy = n + 1; }
    else { Ix = 0; Iy = n - k; }
}

// leaf index of lattice coordinate I (1..n interior, 0 and n+1 on the ring)
__device__ __forceinline__ int leaf_of(int I, int nl)
{
    const int l = (I > 0 ? I - 1 : 0) >> 3;
    return l < nl ? l : nl - 1;
}

// ---------------------------------------------------------------------------
// Pass-1 potential at the 4n ring nodes: near field from the 3x3 leaves
// around the attached boundary leaf (direct log), far field by L2P from
// that leaf's local expansion.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_ring_targets(LeafArgs a, double *__restrict__ phi)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int n = a.n, nl = a.nl;
    if (t >= 4 * n) return;
    int Ix, Iy;
    ring_node(t, n, Ix, Iy);
    const int lx = leaf_of(Ix, nl), ly = leaf_of(Iy, nl);
    const double h = 1.0 / (double)(n + 1);
    double near = 0.0;
    for (int b = -1; b <= 1; ++b)
        for (int c = -1; c <= 1; ++c) {
            const int qx = lx + c, qy = ly + b;
            if (qx < 0 || qy < 0 || qx >= nl || qy >= nl) continue;
            for (int j = 0; j < 8; ++j) {
                const int gy = qy * 8 + j;
                const double dy = (double)(Iy - (gy + 1));
                for (int i = 0; i < 8; ++i) {
                    const int gx = qx * 8 + i;
                    const double dx = (double)(Ix - (gx + 1));
                    near = fma(a.q[(size_t)gy * n + gx], log(h * sqrt(dx * dx + dy * dy)), near);
                }
            }
        }
    double far = 0.0;
    if (a.far) {
        double2 Lc[P];
        local_expansion<P>(a.Lp0, a.Lp1, a.Lp2, a.Lt, a.lv, a.L, lx, ly, Lc);
        const double2 tau = make_double2((Ix - 8 * lx - 4.5) * 0.125, (Iy - 8 * ly - 4.5) * 0.125);
        double2 pw = make_double2(1.0, 0.0);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            far = fma(Lc[k].x, pw.x, fma(-Lc[k].y, pw.y, far));
            pw = cmul(pw, tau);
        }
    }
    phi[t] = -(fma(a.qscale, near, far)) * kInv2Pi;
}

// ---------------------------------------------------------------------------
// Pass 2 (boundary sources): P2M of the ring charges into the boundary
// leaves they attach to.  Interior leaves are never written (stay zero).
// ---------------------------------------------------------------------------
// ring nodes attached to leaf (lx, ly): up to two runs of 8 consecutive
// node indices; returns the number of runs.
__device__ __forceinline__ int attached_runs(int lx, int ly, int n, int nl, int start[2])
{
    int r = 0;
    if (ly == 0) start[r++] = 8 * lx;                        // bottom
    if (lx == nl - 1 && r < 2) start[r++] = n + 8 * ly;        // right
    if (ly == nl - 1 && r < 2) start[r++] = 2 * n + (n - 8 * lx - 8);   // top
    if (lx == 0 && r < 2) start[r++] = 3 * n + (n - 8 * ly - 8);        // left
    return r;
}

template <int P>
__global__ __launch_bounds__(256) void k_p2m_ring(const double *__restrict__ rq,
                                                  double2 *__restrict__ M, int n, int nl)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= nl * nl) return;
    const int lx = idx % nl, ly = idx / nl;
    if (!(lx == 0 || ly == 0 || lx == nl - 1 || ly == nl - 1)) return;
    int start[2];
    // a leaf in a corner touches two sides; with nl == 1 it touches four,
    // which only happens for L = 0, where no multipoles are used
    const int runs = attached_runs(lx, ly, n, nl, start);
    double2 m[P];
#pragma unroll
    for (int k = 0; k < P; ++k) m[k] = make_double2(0.0, 0.0);
    for (int r = 0; r < runs; ++r)
        for (int j = 0; j < 8; ++j) {
            const int t = start[r] + j;
            int Ix, Iy;
            ring_node(t, n, Ix, Iy);
            const double c = rq[t];
            const double2 tau = make_double2((Ix - 8 * lx - 4.5) * 0.125, (Iy - 8 * ly - 4.5) * 0.125);
            m[0].x += c;
            double2 pw = make_double2(1.0, 0.0);
#pragma unroll
            for (int k = 1; k < P; ++k) {
                pw = cmul(pw, tau);
                m[k].x -= c * pw.x / k;
                m[k].y -= c * pw.y / k;
            }
        }
    const int64_t ncell = (int64_t)nl * nl;
#pragma unroll
    for (int k = 0; k < P; ++k) M[k * ncell + idx] = m[k];
}

// Pass 2 at the interior nodes: u += -(1/2pi) [ L2P + direct sum over the
// ring nodes attached to the 3x3 neighbouring leaves ].  Block = 4 leaves
// of 64 points; the leaf's local expansion is built once per leaf.
template <int P>
__global__ __launch_bounds__(256) void k_pass2_leaf(LeafArgs a, const double *__restrict__ rq)
{
    __shared__ double2 sL[4][P];
    const int n = a.n, nl = a.nl;
    const int sub = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int leaf = blockIdx.x * 4 + sub;
    const bool valid = leaf < nl * nl;
    const int lx = valid ? leaf % nl : 0, ly = valid ? leaf / nl : 0;
    if (a.far && j == 0 && valid) {
        double2 Lc[P];
        local_expansion<P>(a.Lp0, a.Lp1, a.Lp2, a.Lt, a.lv, a.L, lx, ly, Lc);
#pragma unroll
        for (int k = 0; k < P; ++k) sL[sub][k] = Lc[k];
    }
    __syncthreads();
    if (!valid) return;
    const int ia = j & 7, jb = j >> 3;
    double far = 0.0;
    if (a.far) {
        const double2 *tp = a.l2p + j * P;
#pragma unroll
        for (int k = 0; k < P; ++k) far = fma(sL[sub][k].x, tp[k].x, fma(-sL[sub][k].y, tp[k].y, far));
    }
    const int gx = lx * 8 + ia, gy = ly * 8 + jb;
    double near = 0.0;
    if (lx <= 1 || ly <= 1 || lx >= nl - 2 || ly >= nl - 2) {
        const double h = 1.0 / (double)(n + 1);
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                const int qx = lx + c, qy = ly + b;
                if (qx < 0 || qy < 0 || qx >= nl || qy >= nl) continue;
                if (!(qx == 0 || qy == 0 || qx == nl - 1 || qy == nl - 1)) continue;
                int start[4], runs = 0;
                if (nl == 1) {
                    start[0] = 0; start[1] = n; start[2] = 2 * n; start[3] = 3 * n;
                    runs = 4;
                } else {
                    runs = attached_runs(qx, qy, n, nl, start);
                }
                for (int r = 0; r < runs; ++r) {
                    const int len = (nl == 1) ? n : 8;
                    for (int e = 0; e < len; ++e) {
                        const int t = start[r] + e;
                        int Ix, Iy;
                        ring_node(t, n, Ix, Iy);
                        const double dx = (double)(gx + 1 - Ix), dy = (double)(gy + 1 - Iy);
                        near = fma(rq[t], log(h * sqrt(dx * dx + dy * dy)), near);
                    }
                }
            }
    }
    a.u[(size_t)gy * n + gx] += -(near + far) * kInv2Pi;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
template <int P>
static void run_m2m(fmm_plan *pl, double2 *M, hipStream_t s)
{
    for (int l = pl->L - 1; l >= 2; --l) {
        const int ncp = 1 << l;
        hipLaunchKernelGGL(k_m2m<P>, dim3((ncp * ncp + 255) / 256), dim3(256), 0, s,
                           M + pl->lv.off[l + 1], M + pl->lv.off[l], pl->tab.m2m, ncp);
    }
}

template <int P>
static int run_upward(fmm_plan *pl, const double *q, double qscale, double2 *M, hipStream_t s)
{
    const int L = pl->L, nl = pl->nl;
    {
        StageTimer t(pl, FMM_STAGE_P2M, s);
        dim3 g1((nl + 31) / 32, nl);
        hipLaunchKernelGGL(k_p2m_grid<P>, g1, dim3(256), 0, s, q, qscale, pl->tab.p2m,
                           M + pl->lv.off[L], (int)pl->n, nl);
    }
    StageTimer t(pl, FMM_STAGE_M2M, s);
    run_m2m<P>(pl, M, s);
    return FMM_OK;
}

template <int P>
static int run_m2l_l2l(fmm_plan *pl, const double2 *M, double2 *const Lp[3], double2 *Lt,
                       const M2LItem *items, int nitems, hipStream_t s, bool timed)
{
    const size_t shm = (size_t)P * 400 * sizeof(double2);
    if (nitems > 0) {
        StageTimer t(pl, timed ? FMM_STAGE_M2L : -1, s);
        hipLaunchKernelGGL(k_m2l<P>, dim3(nitems), dim3(256), shm, s, items, M, Lp[0], Lp[1],
                           Lp[2], pl->lv, pl->tab.hank, pl->tab.m2l_off, pl->tab.m2l_a,
                           pl->tab.m2l_b);
    }
    StageTimer t(pl, timed ? FMM_STAGE_L2L : -1, s);
    for (int l = 2; l <= pl->L - 1; ++l) {
        const int nc = 1 << l;
        hipLaunchKernelGGL(k_l2l<P>, dim3((nc * nc + 255) / 256), dim3(256), 0, s, Lp[0], Lp[1],
                           Lp[2], Lt, pl->lv, l);
    }
    return FMM_OK;
}

template <int P>
static int grid_volume_fmm_p(fmm_plan *pl, const double *q, double qscale, double *u,
                             double *ring_out, hipStream_t s)
{
    const int L = pl->L, nl = pl->nl;
    const bool far = L >= 2;
    if (far) {
        run_upward<P>(pl, q, qscale, pl->ws.M, s);
        run_m2l_l2l<P>(pl, pl->ws.M, pl->ws.Lp, pl->ws.Lt, pl->m2l_items, pl->n_m2l_items, s, true);
    }
    LeafArgs a;
    a.q = q;
    a.qscale = qscale;
    a.u = u;
    a.Lp0 = pl->ws.Lp[0];
    a.Lp1 = pl->ws.Lp[1];
    a.Lp2 = pl->ws.Lp[2];
    a.Lt = pl->ws.Lt;
    a.ktab = pl->tab.ktab;
    a.l2p = pl->tab.l2p;
    a.lv = pl->lv;
    a.n = (int)pl->n;
    a.nl = nl;
    a.L = L;
    a.far = far ? 1 : 0;
    {
        StageTimer t(pl, FMM_STAGE_LEAF, s);
        dim3 gl((nl + 7) / 8, (nl + 7) / 8);
        hipLaunchKernelGGL(k_leaf_grid<P>, gl, dim3(256), 0, s, a);
    }
    if (ring_out) {
        StageTimer t(pl, FMM_STAGE_RING, s);
        hipLaunchKernelGGL(k_ring_targets<P>, dim3((4 * pl->n + 255) / 256), dim3(256), 0, s, a,
                           ring_out);
    }
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

template <int P>
static int grid_ring_source_fmm_p(fmm_plan *pl, double *u, hipStream_t s)
{
    const int L = pl->L, nl = pl->nl;
    const bool far = L >= 2;
    StageTimer t(pl, FMM_STAGE_PASS2, s);
    if (far) {
        hipLaunchKernelGGL(k_p2m_ring<P>, dim3((nl * nl + 255) / 256), dim3(256), 0, s,
                           pl->ring_q, pl->ws.M2 + pl->lv.off[L], (int)pl->n, nl);
        run_m2m<P>(pl, pl->ws.M2, s);
        run_m2l_l2l<P>(pl, pl->ws.M2, pl->ws.Lp2, pl->ws.Lt2, pl->m2l_edge_items,
                       pl->n_m2l_edge_items, s, false);
    }
    LeafArgs a;
    a.q = nullptr;
    a.qscale = 1.0;
    a.u = u;
    a.Lp0 = pl->ws.Lp2[0];
    a.Lp1 = pl->ws.Lp2[1];
    a.Lp2 = pl->ws.Lp2[2];
    a.Lt = pl->ws.Lt2;
    a.ktab = pl->tab.ktab;
    a.l2p = pl->tab.l2p;
    a.lv = pl->lv;
    a.n = (int)pl->n;
    a.nl = nl;
    a.L = L;
    a.far = far ? 1 : 0;
    hipLaunchKernelGGL(k_pass2_leaf<P>, dim3((nl * nl + 3) / 4), dim3(256), 0, s, a, pl->ring_q);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int grid_volume_fmm(fmm_plan *pl, const double *q, double qscale, double *u, double *ring_out,
                    hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, grid_volume_fmm_p, pl, q, qscale, u, ring_out, s);
}

int grid_ring_source_fmm(fmm_plan *pl, double *u, hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, grid_ring_source_fmm_p, pl, u, s);
}

// enable > 64 KB of dynamic LDS for the M2L kernels (gfx950 has 160 KB per CU)
template <int P>
static int m2l_attr_p(fmm_plan *pl)
{
    const int shm = P * 400 * (int)sizeof(double2);
    FMM_HIP(pl, hipFuncSetAttribute((const void *)k_m2l<P>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, shm));
    return FMM_OK;
}

int m2l_kernel_setup(fmm_plan *pl)
{
    FMM_DISPATCH_P(pl->p, m2l_attr_p, pl);
}

}  // namespace fmmprec
