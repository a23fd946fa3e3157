// FMM stages for grid plans on gfx950 (Sec. 5 of arXiv:1308.3339).
//
// The grid is uniform, so every leaf holds the same 8 x 8 point pattern and
// every translation operator depends only on a small integer offset.  The
// stages of one application are:
//   P2P + P2M (Sec. 5.1; 5.3 item 1)  the first kernel: one block per 8x8
//                             leaves stages the q tile once for the near
//                             field (a 3x3-leaf restricted convolution whose
//                             kernel values log(h|d|) are wave-uniform, or an
//                             MFMA contraction in FP32 plans) and the leaf
//                             multipoles
//   M2M    (item 2)           one block per 8x8 tile of cells builds the
//                             multipoles three levels up in LDS, so the
//                             upward pass is ceil((L-2)/3) launches
//   M2L    (item 3)           one launch for all levels; a block is a 16x16
//                             tile of target cells and a third of their
//                             27-entry lists, sources staged in LDS
//   L2L    (item 4)           one block per cell three levels up builds the
//                             local expansions of its 2x2, 4x4, 8x8 descendants
//   L2P    (item 5)           the last sweep over u; in the preconditioner it
//                             also carries the boundary-source pass
//
// Expansions are scaled by the cell width w of their level (M~_k = M_k/w^k,
// L~_k = L_k w^k), which makes M2M, M2L and L2L level independent.
#include <algorithm>
#include <utility>
#include <vector>

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

__device__ __forceinline__ void cmac(float2 &acc, float2 a, float2 b)
{
    acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
    acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

// real type -> complex pair type
template <typename R> struct Cplx;
template <> struct Cplx<double> { using T = double2; };
template <> struct Cplx<float> { using T = float2; };

__device__ __forceinline__ double wave_sum(double a)
{
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    return a;
}

// Block-wide LDS staging for 256-thread blocks, split in two halves:
// fetch() loads elements t = tid + 256 r (t < cnt) of a gather into
// registers, put() hands them to a store functor.  Kernels fetch every table
// and tile before storing any of them, so a block waits for one memory round
// trip rather than one per loop trip.
constexpr int rounds256(int cnt) { return (cnt + 255) / 256; }

template <int R, typename T, typename F>
__device__ __forceinline__ void fetch(T (&v)[R], int cnt, F src)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = threadIdx.x + 256 * r;
        if (t < cnt) v[r] = src(t);
    }
}

template <int R, typename T, typename F>
__device__ __forceinline__ void put(const T (&v)[R], int cnt, F dst)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = threadIdx.x + 256 * r;
        if (t < cnt) dst(t, v[r]);
    }
}

// ---------------------------------------------------------------------------
// Upward pass.
// m2m_tile: parents of a cw x cw child tile held in LDS as [k][cw*cw];
// A = M2M table [4 quadrants][P][P] (lower triangular), quadrant
// qd = 2*(child y parity) + (child x parity).
// ---------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void m2m_tile(const double2 *__restrict__ sA,
                                         const double2 *__restrict__ child,
                                         double2 *__restrict__ parent, int cw)
{
    // cw is a power of two: indices by shifts
    const int pw = cw >> 1, np = pw * pw, nch = cw * cw, lpw = __builtin_ctz(pw);
    for (int t = threadIdx.x; t < np * P; t += blockDim.x) {
        const int nn = t >> (2 * lpw), pc = t & (np - 1);
        const int px = pc & (pw - 1), py = pc >> lpw;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            const int ci = (2 * py + (qd >> 1)) * cw + 2 * px + (qd & 1);
            const double2 *Ar = sA + (qd * P + nn) * P;
#pragma unroll
            for (int k = 0; k < P; ++k)
                if (k <= nn) cmac(acc, Ar[k], child[k * nch + ci]);
        }
        parent[nn * np + pc] = acc;
    }
}

// tile (LDS [k][tw*tw]) -> level array at origin (x0, y0)
template <int P>
__device__ __forceinline__ void store_tile(const double2 *__restrict__ src, double2 *__restrict__ Ml,
                                           int nc, int x0, int y0, int tw)
{
    const int cnt = tw * tw, ltw = __builtin_ctz(tw);   // tw is a power of two
    const int64_t ncell = (int64_t)nc * nc;
    for (int t = threadIdx.x; t < P * cnt; t += blockDim.x) {
        const int k = t >> (2 * ltw), c = t & (cnt - 1);
        Ml[k * ncell + (int64_t)(y0 + (c >> ltw)) * nc + x0 + (c & (tw - 1))] = src[t];
    }
}

// multipoles of a tile three more levels up, each level stored to global
template <int P>
__device__ __forceinline__ void m2m_chain(const double2 *sA, double2 *s0, double2 *s1, double2 *s2,
                                          double2 *s3, double2 *__restrict__ M, const LevelInfo &lv,
                                          int l, int tw, int x0, int y0)
{
    double2 *cur = s0;
    double2 *bufs[3] = {s1, s2, s3};
    for (int st = 0; st < 3 && l - 1 >= 2 && tw >= 2; ++st) {
        m2m_tile<P>(sA, cur, bufs[st], tw);
        __syncthreads();
        tw >>= 1;
        --l;
        x0 >>= 1;
        y0 >>= 1;
        store_tile<P>(bufs[st], M + lv.off[l], 1 << l, x0, y0, tw);
        cur = bufs[st];
    }
}


// M2M from level l_in three levels up, one 8x8 tile of level-l_in cells per
// block.
template <int P>
__global__ __launch_bounds__(256) void k_m2m_up(double2 *__restrict__ M,
                                                const double2 *__restrict__ A, LevelInfo lv,
                                                int l_in, RhsSet rh)
{
    if (!rhs_active(rh, blockIdx.z)) return;
    M += blockIdx.z * rh.se;
    __shared__ double2 sA[4 * P * P];
    __shared__ double2 s0[P * 64], s1[P * 16], s2[P * 4], s3[P];
    const int nc = 1 << l_in, tw = nc < 8 ? nc : 8, nt = nc / tw;
    const int tx = blockIdx.x % nt, ty = blockIdx.x / nt;
    const int x0 = tx * tw, y0 = ty * tw, cnt = tw * tw;
    const int64_t ncell = (int64_t)nc * nc;
    const double2 *Ml = M + lv.off[l_in];
    const int ltw = __builtin_ctz(tw);
    {
        double2 va[rounds256(4 * P * P)], vs[rounds256(P * 64)];
        fetch(va, 4 * P * P, [&](int t) { return A[t]; });
        fetch(vs, P * cnt, [&](int t) {
            const int k = t >> (2 * ltw), c = t & (cnt - 1);
            return Ml[k * ncell + (int64_t)(y0 + (c >> ltw)) * nc + x0 + (c & (tw - 1))];
        });
        put(va, 4 * P * P, [&](int t, double2 x) { sA[t] = x; });
        put(vs, P * cnt, [&](int t, double2 x) { s0[t] = x; });
    }
    __syncthreads();
    m2m_chain<P>(sA, s0, s1, s2, s3, M, lv, l_in, tw, x0, y0);
}

// ---------------------------------------------------------------------------
// M2L for all levels 2..L in one launch.
// Scaled Hankel form of Sec. 5.3 item 3: with d^ = offset in cell widths,
//   L~_n = a_n sum_k H_{n+k} M'_k,  a_n = (-1)^n/n!,
//   M'_0 = -M~_0, M'_k = M~_k/(k-1)!,
//   H_0 = -(log|d^| + log w), H_m = (m-1)!/d^^m.
// A block is a 16x16 tile of target cells (the whole level if it is
// smaller) and share item.part of nsplit of the interaction lists (its sums
// go to part item.part of Lm, lm_part apart; the downward pass adds the
// parts), with 12 waves: wave w serves parity class w&3 (cells that share
// one list shape, so the offset and its Hankel generators are wave-uniform)
// and third w>>2 of the block's share of the class's nlist-entry list (27
// entries with the list rule, more with a MAC theta).  Splitting the lists
// gives small trees enough blocks: a 1024^2 grid has 87 tiles for 256
// compute units.  Sources (the tile plus a halo of 2K cells, 20x20 for
// K = 1) are staged once in LDS, a thread per source cell with its P
// coefficients (64 KB at p = 10, so two blocks share a compute unit), split
// by parity, each parity sub-grid column-major: a 16-byte read of 8 columns
// x 2 rows of a wave's cells then puts its 16 lanes on 16 distinct 16-byte
// bank groups (column stride RH = 10, even, and rows one apart); the three
// thirds are summed in LDS in a fixed order.  R is the arithmetic type of the translation (double, or
// float for the FP32 variant; the level-scaled expansions and generators
// stay far inside FP32 range for p <= 20), inputs and outputs are FP64.
// hank holds the generators in list order ([class][entry][2P-1]), so the
// address of an entry's generators does not wait for its offset to load.
// ---------------------------------------------------------------------------
constexpr int kM2LGroups = 3;   // list groups per parity class in a k_m2l block
constexpr int kM2LThreads = 256 * kM2LGroups;

template <int P, typename R>
__global__ __launch_bounds__(kM2LThreads) void k_m2l(const M2LItem *__restrict__ items,
                                             const double2 *__restrict__ M,
                                             double2 *__restrict__ Lm, int64_t lm_part,
                                             int nsplit, LevelInfo lv,
                                             const typename Cplx<R>::T *__restrict__ hank,
                                             const int4 *__restrict__ offs,
                                             const double *__restrict__ a_n,
                                             const double *__restrict__ b_k, int nlist,
                                             int halo, RhsSet rh)
{
    using C = typename Cplx<R>::T;
    if (!rhs_active(rh, blockIdx.z)) return;
    M += blockIdx.z * rh.se;
    Lm += blockIdx.z * rh.se;
    extern __shared__ __align__(16) unsigned char sm_raw[];
    C *sm = reinterpret_cast<C *>(sm_raw);   // [P][RW*RW] parity split; later [P][256] reduction
    const M2LItem it = items[blockIdx.x];
    const int l = it.level, nc = 1 << l;
    const int tw = nc < 16 ? nc : 16;
    const int RW = tw + 2 * halo, RH = RW >> 1, SUB = RH * RH, RR = RW * RW;
    const int64_t ncell = (int64_t)nc * nc;
    const double2 *Ml = M + lv.off[l];
    // stage: a thread takes one source cell and its P coefficients (one
    // division per cell, P loads in flight)
    for (int r = threadIdx.x; r < RR; r += kM2LThreads) {
        const int sy = r / RW, sx = r - sy * RW;
        const int gx = it.tx0 - halo + sx, gy = it.ty0 - halo + sy;
        const bool in = gx >= 0 && gx < nc && gy >= 0 && gy < nc;
        const int64_t gi = in ? (int64_t)gy * nc + gx : 0;
        double2 v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = in ? Ml[k * ncell + gi] : make_double2(0.0, 0.0);
        const int si = ((sy & 1) * 2 + (sx & 1)) * SUB + (sx >> 1) * RH + (sy >> 1);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double bk = b_k[k];
            C c;
            c.x = (R)(v[k].x * bk);
            c.y = (R)(v[k].y * bk);
            sm[k * RR + si] = c;
        }
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int cls = wave & 3, grp = wave >> 2;
    const int px = cls & 1, py = cls >> 1;
    const int ltx = 2 * (lane & 7) + px, lty = 2 * (lane >> 3) + py;
    const bool active = ltx < tw && lty < tw;
    C acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k].x = acc[k].y = (R)0;
    const R logw = (R)lv.logw[l];
    // this block's share of the list: entries [lo, lo + cnt), in groups
    const int per = (nlist + nsplit - 1) / nsplit;
    const int lo = it.part * per, cnt = max(0, min(per, nlist - lo));
    const int chunk = (cnt + kM2LGroups - 1) / kM2LGroups;
    const int4 *ol = offs + cls * nlist + lo + grp * chunk;
    const C *Hl = hank + (size_t)(cls * nlist + lo + grp * chunk) * (2 * P - 1);
    const int nown = max(0, min(chunk, cnt - grp * chunk));
    if (active) {
        for (int o = 0; o < nown; ++o) {
            const int4 od = ol[o];
            const C *H = Hl + o * (2 * P - 1);
            const int sx = ltx + od.x + halo, sy = lty + od.y + halo;
            const int sidx = ((sy & 1) * 2 + (sx & 1)) * SUB + (sx >> 1) * RH + (sy >> 1);
            C m[P];
#pragma unroll
            for (int k = 0; k < P; ++k) m[k] = sm[k * RR + sidx];
            // anti-diagonal order: each generator H_s is used by all (n, k), n+k = s
#pragma unroll
            for (int s = 0; s < 2 * P - 1; ++s) {
                C h = H[s];
                if (s == 0) h.x -= logw;
#pragma unroll
                for (int nn = (s < P ? 0 : s - P + 1); nn <= (s < P ? s : P - 1); ++nn)
                    cmac(acc[nn], h, m[s - nn]);
            }
        }
    }
    // sum the groups in order: ((group 0 + group 1) + group 2) + ...
    const int slot = cls * 64 + lane;
    for (int g = 1; g < kM2LGroups; ++g) {
        __syncthreads();
        if (grp == g && active) {
#pragma unroll
            for (int k = 0; k < P; ++k) sm[k * 256 + slot] = acc[k];
        }
        __syncthreads();
        if (grp == 0 && active) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const C v = sm[k * 256 + slot];
                acc[k].x += v.x;
                acc[k].y += v.y;
            }
        }
    }
    if (grp != 0 || !active) return;
    const int tx = it.tx0 + ltx, ty = it.ty0 + lty;
    double2 *out = Lm + it.part * lm_part + lv.off[l];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double an = a_n[k];
        out[k * ncell + (int64_t)ty * nc + tx] = make_double2(an * (double)acc[k].x, an * (double)acc[k].y);
    }
}

// ---------------------------------------------------------------------------
// Downward pass: one block per cell at level r builds the local expansions
// of its descendants at levels r+1 .. r+m (m <= 3):
//   L~child_n = sum_{k>=n} B[qd][n][k] L~parent_k + (M2L sum of the child),
//   B[qd][n][k] = C(k,n) c^(k-n) 2^-n, c = (child - parent centre)/w_parent.
// With top = 1 the root is a level-2 cell, whose expansion is its M2L sum
// alone (lists start at level 2), and is written too.  All M2L sums the
// block needs are fetched into LDS up front (one memory round trip).
// ---------------------------------------------------------------------------
// Shared body of the downward chain.  The block owns cell (rx, ry) of level
// r, whose expansion is in buf0[0..P).  Levels r+1..r+m are built in LDS
// (and stored to Lt when Lt != nullptr); returns the buffer that holds the
// deepest level, laid out [k][tw*tw] with tw = 2^m.
// The block's own expansion is read from top[k * top_stride] (k < P) in the
// same round trip as the tables and M2L sums, and also stored to top_out when
// that is not null.  With top == nullptr it is built instead from the M2L
// sums of its ancestors at levels 2..r (r <= 5), fetched in the same round
// trip: L~_2 = M2L sum of the level-2 ancestor, then L~_l = B L~_(l-1) + M2L
// sum, the same chain the launches above it would compute, so that the
// levels above r need no launch of their own.
constexpr int kMaxAncestorLevel = 5;

template <int P>
__device__ __forceinline__ double2 *down_levels(const double2 *__restrict__ Lm, int nsplit,
                                                      int64_t lm_part,
                                                      double2 *__restrict__ Lt,
                                                      const double2 *__restrict__ B,
                                                      const LevelInfo &lv, int r, int m, int rx,
                                                      int ry, double2 *sB, double2 *sm2l,
                                                      double2 *buf0, double2 *buf1,
                                                      const double2 *__restrict__ top,
                                                      int64_t top_stride, bool top_m2l,
                                                      double2 *__restrict__ top_out,
                                                      double2 *sanc)
{
    const bool anc = top == nullptr;
    // the M2L sums are held in nsplit parts lm_part apart (one per share of
    // the interaction lists): part 0 is stored, later parts are added in
    // order, each part in one round trip (a thread adds into the LDS words
    // it wrote itself, so the parts need no barrier between them)
    for (int pp = 0; pp < nsplit; ++pp) {
        const double2 *__restrict__ Lp = Lm + pp * lm_part;
        const bool first = pp == 0;
        const bool with_top = !anc && (first || top_m2l);
        const double2 *__restrict__ tp = top_m2l ? top + pp * lm_part : top;
        // M2L sum k of the level-(2 + j) ancestor, t = j P + k
        auto anc_sum = [&](int t) {
            const int j = t / P, k = t - j * P, l = 2 + j, nc = 1 << l;
            const int ax = rx >> (r - l), ay = ry >> (r - l);
            return Lp[lv.off[l] + k * (int64_t)nc * nc + (int64_t)ay * nc + ax];
        };
        double2 va[rounds256((kMaxAncestorLevel - 1) * P)];
        fetch(va, anc ? (r - 1) * P : 0, anc_sum);
        auto m2l_sum = [&](int st, int t) {
            const int l = r + st, tw = 1 << st, nc = 1 << l;
            const int nn = t >> (2 * st), c = t & (tw * tw - 1);
            return Lp[lv.off[l] + nn * (int64_t)nc * nc + (int64_t)(ry * tw + (c >> st)) * nc +
                      rx * tw + (c & (tw - 1))];
        };
        double2 vb[rounds256(4 * P * P)], vt[1], v1[rounds256(4 * P)], v2[rounds256(16 * P)],
            v3[rounds256(64 * P)];
        fetch(vb, first ? 4 * P * P : 0, [&](int t) { return B[t]; });
        fetch(vt, with_top ? P : 0, [&](int t) { return tp[t * top_stride]; });
        fetch(v1, m >= 1 ? 4 * P : 0, [&](int t) { return m2l_sum(1, t); });
        fetch(v2, m >= 2 ? 16 * P : 0, [&](int t) { return m2l_sum(2, t); });
        fetch(v3, m >= 3 ? 64 * P : 0, [&](int t) { return m2l_sum(3, t); });
        auto st = [first](double2 &d, double2 x) {
            if (first) {
                d = x;
            } else {
                d.x += x.x;
                d.y += x.y;
            }
        };
        put(vb, first ? 4 * P * P : 0, [&](int t, double2 x) { sB[t] = x; });
        put(va, anc ? (r - 1) * P : 0, [&](int t, double2 x) { st(sanc[t], x); });
        put(vt, with_top ? P : 0, [&](int t, double2 x) { st(buf0[t], x); });
        put(v1, m >= 1 ? 4 * P : 0, [&](int t, double2 x) { st(sm2l[(t >> 2) * 84 + (t & 3)], x); });
        put(v2, m >= 2 ? 16 * P : 0, [&](int t, double2 x) { st(sm2l[(t >> 4) * 84 + 4 + (t & 15)], x); });
        put(v3, m >= 3 ? 64 * P : 0, [&](int t, double2 x) { st(sm2l[(t >> 6) * 84 + 20 + (t & 63)], x); });
    }
    // the root's whole expansion, by the threads that summed it (t < P <= 256)
    if (top_out && !anc && (int)threadIdx.x < P) top_out[threadIdx.x * top_stride] = buf0[threadIdx.x];
    __syncthreads();
    if (anc) {
        // down the ancestors, one coefficient per thread, into buf0
        const double2 *cur = sanc;
        for (int l = 3; l <= r; ++l) {
            const int ax = rx >> (r - l), ay = ry >> (r - l), qd = (ay & 1) * 2 + (ax & 1);
            double2 *out = l == r ? buf0 : buf1 + (l & 1) * P;
            if (threadIdx.x < P) {
                const int nn = threadIdx.x;
                double2 acc = sanc[(l - 2) * P + nn];
                const double2 *Br = sB + (qd * P + nn) * P;
#pragma unroll
                for (int k = 0; k < P; ++k)
                    if (k >= nn) cmac(acc, Br[k], cur[k]);
                out[nn] = acc;
            }
            __syncthreads();
            cur = out;
        }
        if (r == 2 && threadIdx.x < P) buf0[threadIdx.x] = sanc[threadIdx.x];
        __syncthreads();
    }
    double2 *prev = buf0;
    int pw = 1;
    for (int st = 1; st <= m; ++st) {
        const int l = r + st, tw = 1 << st, nc = 1 << l, cnt = tw * tw;
        const int base = ((1 << (2 * st)) - 4) / 3;
        const int64_t ncell = (int64_t)nc * nc;
        double2 *next = (st & 1) ? buf1 : buf0;
        const int pcnt = pw * pw;
        for (int t = threadIdx.x; t < P * cnt; t += blockDim.x) {
            const int nn = t >> (2 * st), c = t & (cnt - 1);
            const int cx = c & (tw - 1), cy = c >> st;
            const int pc = (cy >> 1) * pw + (cx >> 1), qd = (cy & 1) * 2 + (cx & 1);
            double2 acc = sm2l[nn * 84 + base + c];
            const double2 *Br = sB + (qd * P + nn) * P;
#pragma unroll
            for (int k = 0; k < P; ++k)
                if (k >= nn) cmac(acc, Br[k], prev[k * pcnt + pc]);
            next[t] = acc;
            if (Lt) Lt[lv.off[l] + nn * ncell + (int64_t)(ry * tw + cy) * nc + rx * tw + cx] = acc;
        }
        __syncthreads();
        prev = next;
        pw = tw;
    }
    return prev;
}

// root: 1 = the root is a level-2 cell (its expansion is its M2L sum, also
// stored), 0 = read the root's expansion from Lt, 2 = build it from the
// ancestors (r <= 5).  The M2L sums are the nsplit parts of Lm, lm_part apart.
template <int P>
__global__ __launch_bounds__(256) void k_down(const double2 *__restrict__ Lm, int nsplit,
                                              int64_t lm_part, double2 *__restrict__ Lt,
                                              const double2 *__restrict__ B, LevelInfo lv, int r,
                                              int m, int root, RhsSet rh)
{
    if (!rhs_active(rh, blockIdx.z)) return;
    Lm += blockIdx.z * rh.se;
    Lt += blockIdx.z * rh.se;
    __shared__ double2 sB[4 * P * P];
    __shared__ double2 sm2l[P * 84];          // M2L sums of the 4 + 16 + 64 descendants
    __shared__ double2 buf0[P * 64], buf1[P * 64];
    __shared__ double2 sanc[(kMaxAncestorLevel - 1) * P];
    const int nr = 1 << r;
    const int rx = blockIdx.x & (nr - 1), ry = blockIdx.x >> r;
    const int64_t gi = lv.off[r] + (int64_t)ry * nr + rx;
    const double2 *top = root == 2 ? nullptr : (root == 1 ? Lm : Lt) + gi;
    down_levels<P>(Lm, nsplit, lm_part, Lt, B, lv, r, m, rx, ry, sB, sm2l, buf0, buf1, top,
                   (int64_t)nr * nr, root == 1, root == 1 ? Lt + gi : nullptr, sanc);
}

// ---------------------------------------------------------------------------
// Leaf stage for grid plans, the first kernel of an application:
//   u = -(1/2pi) qscale * sum_{3x3 leaves} q_j T(d_ij)     (P2P, Sec. 5.1)
//   M~_k(leaf) = qscale * sum_{j in leaf} W[k][j] q_j       (P2M, Sec. 5.3)
// T(d) = log(h|d|) for lattice offsets d != 0 and log(eps h) for d = 0 (the
// regularised self term); W[0][j] = 1, W[k][j] = -tau_j^k / k with tau_j the
// point's offset from the leaf centre in leaf widths.  Both read the q tile
// the block stages once.  The far field is added later by k_far_l2p.  Block = 8x8 leaves; lane = leaf; wave w of 8
// serves target row w of every leaf (8 targets per lane).  For a fixed
// source position all lanes need the same T values, so T rows are read with
// scalar loads and broadcast, and the q tile sits in LDS as [pos][leaf].
// Launch bounds of six waves per SIMD (at most 80 VGPRs: three blocks per CU).
// ---------------------------------------------------------------------------
// LDS layout of the 10x10-leaf q tile of the leaf kernels.  Source position
// pos (0..63) of leaf (row r, col c) sits at
//   (pos / 4) * 400 + r * 40 + (pos % 4) * 10 + c,
// i.e. rows are 40 elements apart and hold the columns of four positions
// side by side.  A wave reads one position of an 8x8 window of leaves;
// with the row stride = 8 mod 32 doubles those 64 elements fall on distinct
// banks (64 x 4-byte banks, FP64 in half-waves or FP32 in one pass), where
// a stride of 10 left half the LDS cycles as bank conflicts.
__device__ __forceinline__ constexpr int leaf_tile_idx(int pos, int r, int c)
{
    return (pos >> 2) * 400 + r * 40 + (pos & 3) * 10 + c;
}

struct LeafArgs {
    RhsSet rh;            // right-hand side blockIdx.z: strides and active mask
    const double *q;
    double qscale;
    double *u;
    const double2 *Lt;    // local expansions (leaf level used)
    const double *ktab;   // [31][31]
    const double *rtab;   // [17][17]
    const double2 *l2p;   // [64][P]
    double2 *M;           // leaf multipoles written by the FP64 leaf kernel (null: no P2M)
    const double2 *p2m;   // [P][64]
    LevelInfo lv;
    int n, nl, L, far;
    // near set (Sec. 5.2): radius K leaves; leaves (a, b) with |a| <= kx(|b|)
    // are near, kx(b) + 1 packed in 4 bits each (near_kx); rtab side rs = 8K + 9
    // (ktab side 16K + 15)
    int K, kxp, rs;
};

__device__ __forceinline__ int near_kx(int kxp, int b)
{
    return ((kxp >> (4 * b)) & 15) - 1;
}

// The arrays of right-hand side blockIdx.z (on = false when that right-hand
// side is inactive: the whole block leaves).  The kernels keep a itself in
// the kernel arguments and take these four pointers from here.
struct LeafPtrs {
    bool on;
    const double *q;
    double *u;
    double2 *M;
    const double2 *Lt;
};
__device__ __forceinline__ LeafPtrs rhs_ptrs(const LeafArgs &a)
{
    const int r = blockIdx.z;
    LeafPtrs p;
    p.on = rhs_active(a.rh, r);
    p.q = a.q ? a.q + r * a.rh.sv : nullptr;
    p.u = a.u ? a.u + r * a.rh.sv : nullptr;
    p.M = a.M ? a.M + r * a.rh.se : nullptr;
    p.Lt = a.Lt ? a.Lt + r * a.rh.se : nullptr;
    return p;
}

template <int P>
__global__ __launch_bounds__(512, 6) void k_leaf_grid(LeafArgs a)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on) return;
    __shared__ double sq[6400];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, nl = a.nl;
    const int TX0 = blockIdx.x * 8, TY0 = blockIdx.y * 8;
    const int X0 = (TX0 - 1) * 8, Y0 = (TY0 - 1) * 8;
    {
        // all 13 loads of a thread are issued before any LDS store
        double v[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const int e = tid + 512 * i;
            const int yy = e / 80, xx = e - yy * 80;
            const int gx = X0 + xx, gy = Y0 + yy;
            v[i] = (e < 6400 && gx >= 0 && gx < n && gy >= 0 && gy < n) ? pp.q[(size_t)gy * n + gx] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const int e = tid + 512 * i;
            const int yy = e / 80, xx = e - yy * 80;
            if (e < 6400) sq[leaf_tile_idx((yy & 7) * 8 + (xx & 7), yy >> 3, xx >> 3)] = v[i];
        }
    }
    __syncthreads();
    const int lx = lane & 7, ly = lane >> 3;
    const int gLx = TX0 + lx, gLy = TY0 + ly;
    const bool active = gLx < nl && gLy < nl;
    const int ty = wave;
    const int cleaf = leaf_tile_idx(0, ly + 1, lx + 1);
    double acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = 0.0;
    const double *__restrict__ kt = a.ktab;
    for (int oy = -1; oy <= 1; ++oy) {
        for (int sy = 0; sy < 8; ++sy) {
            const double *T0 = kt + (8 * oy + sy - ty + 15) * 31 + 8;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                double w0[15];
#pragma unroll
                for (int c = 0; c < 15; ++c) w0[c] = T0[8 * ox + c];
                const int sl = cleaf + oy * 40 + ox;
#pragma unroll
                for (int sx = 0; sx < 8; ++sx) {
                    const double v = sq[leaf_tile_idx(sy * 8 + sx, 0, 0) + sl];
#pragma unroll
                    for (int tx = 0; tx < 8; ++tx) acc[tx] = fma(w0[sx - tx + 7], v, acc[tx]);
                }
            }
        }
    }
    if (pp.M) {
        // P2M: wave w computes coefficients w, w + 8, ... of the 64 leaves
        const int64_t ncell = (int64_t)nl * nl, cell = (int64_t)gLy * nl + gLx;
        double2 *Ml = pp.M + a.lv.off[a.L];
        for (int k = wave; k < P; k += 8) {
            const double2 *__restrict__ Wk = a.p2m + k * 64;
            double mx = 0.0, my = 0.0;
#pragma unroll 8
            for (int j = 0; j < 64; ++j) {
                const double v = sq[leaf_tile_idx(j, 0, 0) + cleaf];
                const double2 w = Wk[j];
                mx = fma(w.x, v, mx);
                my = fma(w.y, v, my);
            }
            if (active) Ml[k * ncell + cell] = make_double2(mx * a.qscale, my * a.qscale);
        }
    }
    if (!active) return;
    const double qs = -a.qscale * kInv2Pi;
    double *ur = pp.u + (size_t)(gLy * 8 + ty) * n + gLx * 8;
#pragma unroll
    for (int t = 0; t < 8; ++t) ur[t] = qs * acc[t];
}

// Leaf stage with the near set of a MAC theta (Sec. 5.2): on the uniform tree
// the dual tree traversal's P2P pairs of a leaf are the leaves of the
// lattice disk |d|^2 <= 2/theta^2, radius K <= 4 leaves, instead of the 3x3
// block.  Same organisation as k_leaf_grid (block = 8x8 leaves, lane = leaf,
// wave = target row, T rows by scalar loads) with the (8+2K)^2-leaf q tile in
// LDS and, per row of leaf offsets, the column range from the packed kx.
// Tile layout as leaf_tile_idx, with a column slot CW >= 8 + 2K chosen so that
// the row stride 4 CW is 8 or 24 mod 32 doubles (distinct banks for the 8x8
// window a wave reads).
template <int K>
struct WideTile {
    static constexpr int TW = 8 + 2 * K;
    static constexpr int CW = K <= 3 ? 14 : 18;
    static constexpr int RS = 4 * CW;
    static constexpr int PS = TW * RS;
    static constexpr int SIZE = 16 * PS;
    __device__ static constexpr int idx(int pos, int r, int c)
    {
        return (pos >> 2) * PS + r * RS + (pos & 3) * CW + c;
    }
};

template <int P, int K>
__global__ __launch_bounds__(512) void k_leaf_wide(LeafArgs a)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on) return;
    using W = WideTile<K>;
    __shared__ double sq[W::SIZE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, nl = a.nl;
    const int TX0 = blockIdx.x * 8, TY0 = blockIdx.y * 8;
    const int X0 = (TX0 - K) * 8, Y0 = (TY0 - K) * 8;
    constexpr int PW = 8 * W::TW, NE = PW * PW, NB = 13;
    for (int base = 0; base < NE; base += 512 * NB) {
        double v[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = base + tid + 512 * i;
            const int yy = e / PW, xx = e - yy * PW;
            const int gx = X0 + xx, gy = Y0 + yy;
            v[i] = (e < NE && gx >= 0 && gx < n && gy >= 0 && gy < n) ? pp.q[(size_t)gy * n + gx] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = base + tid + 512 * i;
            const int yy = e / PW, xx = e - yy * PW;
            if (e < NE) sq[W::idx((yy & 7) * 8 + (xx & 7), yy >> 3, xx >> 3)] = v[i];
        }
    }
    __syncthreads();
    const int lx = lane & 7, ly = lane >> 3;
    const int gLx = TX0 + lx, gLy = TY0 + ly;
    const bool active = gLx < nl && gLy < nl;
    const int ty = wave;
    const int cleaf = W::idx(0, ly + K, lx + K);
    constexpr int KC = 8 * K + 7, KS = 2 * KC + 1;
    double acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = 0.0;
    const double *__restrict__ kt = a.ktab;
    for (int oy = -K; oy <= K; ++oy) {
        const int kxo = near_kx(a.kxp, oy < 0 ? -oy : oy);
        for (int sy = 0; sy < 8; ++sy) {
            const double *T0 = kt + (8 * oy + sy - ty + KC) * KS + KC - 7;
            for (int ox = -kxo; ox <= kxo; ++ox) {
                double w0[15];
#pragma unroll
                for (int c = 0; c < 15; ++c) w0[c] = T0[8 * ox + c];
                const int sl = cleaf + oy * W::RS + ox;
#pragma unroll
                for (int sx = 0; sx < 8; ++sx) {
                    const double v = sq[W::idx(sy * 8 + sx, 0, 0) + sl];
#pragma unroll
                    for (int tx = 0; tx < 8; ++tx) acc[tx] = fma(w0[sx - tx + 7], v, acc[tx]);
                }
            }
        }
    }
    if (pp.M) {
        const int64_t ncell = (int64_t)nl * nl, cell = (int64_t)gLy * nl + gLx;
        double2 *Ml = pp.M + a.lv.off[a.L];
        for (int k = wave; k < P; k += 8) {
            const double2 *__restrict__ Wk = a.p2m + k * 64;
            double mx = 0.0, my = 0.0;
#pragma unroll 8
            for (int j = 0; j < 64; ++j) {
                const double v = sq[W::idx(j, 0, 0) + cleaf];
                const double2 w = Wk[j];
                mx = fma(w.x, v, mx);
                my = fma(w.y, v, my);
            }
            if (active) Ml[k * ncell + cell] = make_double2(mx * a.qscale, my * a.qscale);
        }
    }
    if (!active) return;
    const double qs = -a.qscale * kInv2Pi;
    double *ur = pp.u + (size_t)(gLy * 8 + ty) * n + gLx * 8;
#pragma unroll
    for (int t = 0; t < 8; ++t) ur[t] = qs * acc[t];
}

// FP32 variant of the leaf stage (precision variant of the preconditioner) on
// the matrix cores.  On the grid the near field is a Toeplitz contraction:
// for each of the 9 leaf offsets o, U(target pos t, leaf) += K_o[t][s] *
// Q(source pos s, leaf + o) with K_o[t][s] = T(8 o + s_xy - t_xy), so it maps
// onto v_mfma_f32_16x16x4f32: M = 64 target positions (4 tiles), N = 16
// leaves per wave, K = 64 source positions per offset (16 steps).  The FP32
// products of one offset are summed in the matrix core (64 terms) and folded
// into FP64 accumulators, so FP32 rounding stays at the level of one 64-term
// sum.  P2M is the same contraction with the P2M weights as A rows (2k: Re,
// 2k+1: Im) and the centre leaves as B.  Block = 8x8 target leaves, wave w =
// leaves 16w..16w+15 (rows 2w, 2w+1).  LDS: the 10x10-leaf q tile in FP32 at
// (pos/4)*453 + row*136 + (pos%4)*80 + col, which puts the 64 lanes of a B
// read (4 positions x 16 leaves) on distinct banks, and T with rows 48 apart.
// MFMA lane layout (16x16x4f32): A[l%16][l/16], B[l/16][l%16],
// D[4(l/16)+i][l%16].
__device__ __forceinline__ constexpr int mq_idx(int pos, int r, int c)
{
    return (pos >> 2) * 453 + r * 136 + (pos & 3) * 80 + c;
}

template <int P>
__global__ __launch_bounds__(256) void k_leaf_mfma32(LeafArgs a, const float *__restrict__ kt32,
                                                     const float *__restrict__ w32)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on) return;
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int MTP = (2 * P + 15) / 16;      // P2M row tiles
    __shared__ float sq[mq_idx(63, 9, 9) + 1];
    __shared__ float st[31 * 48];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, nl = a.nl;
    const int TX0 = blockIdx.x * 8, TY0 = blockIdx.y * 8;
    const int X0 = (TX0 - 1) * 8, Y0 = (TY0 - 1) * 8;
    {
        float v[25], tv[4];
#pragma unroll
        for (int i = 0; i < 25; ++i) {
            const int e = tid + 256 * i;
            const int yy = e / 80, xx = e - yy * 80;
            const int gx = X0 + xx, gy = Y0 + yy;
            v[i] = (gx >= 0 && gx < n && gy >= 0 && gy < n) ? (float)pp.q[(size_t)gy * n + gx] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            tv[i] = e < 961 ? kt32[e] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 25; ++i) {
            const int e = tid + 256 * i;
            const int yy = e / 80, xx = e - yy * 80;
            sq[mq_idx((yy & 7) * 8 + (xx & 7), yy >> 3, xx >> 3)] = v[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            if (e < 961) st[(e / 31) * 48 + e % 31] = tv[i];
        }
    }
    __syncthreads();
    const int g = lane >> 4, m16 = lane & 15;
    const int nloc = 16 * wave + m16;              // target leaf of this lane's B column
    const int lx = nloc & 7, ly = nloc >> 3;
    // A operand of lane: target t = 16 mt + m16 -> tx = lane & 7, ty = 2 mt + ((lane >> 3) & 1);
    // source s = 4 kk + g -> sx = 4 (kk & 1) + g, sy = kk >> 1
    const int abase = (15 - ((lane >> 3) & 1)) * 48 + 15 + g - (lane & 7);
    const int bbase = (ly + 1) * 136 + g * 80 + lx + 1;
    double acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mt][i] = 0.0;
#pragma unroll 1
    for (int o = 0; o < 9; ++o) {
        const int oy = o / 3 - 1, ox = o % 3 - 1;
        f4 c[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) c[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        const float *Ab = st + abase + 8 * oy * 48 + 8 * ox;
        const float *Bb = sq + bbase + oy * 136 + ox;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const float b = Bb[kk * 453];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                c[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    Ab[((kk >> 1) - 2 * mt) * 48 + 4 * (kk & 1)], b, c[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[mt][i] += (double)c[mt][i];
    }
    // P2M: rows of w32 against the centre leaves
    f4 pm[MTP];
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt) pm[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    if (pp.M) {
        const float *Bb = sq + bbase;
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const float b = Bb[kk * 453];
#pragma unroll
            for (int mt = 0; mt < MTP; ++mt)
                pm[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(w32[(16 * mt + m16) * 64 + 4 * kk + g], b,
                                                              pm[mt], 0, 0, 0);
        }
    }
    const int gLx = TX0 + lx, gLy = TY0 + ly;
    if (gLx >= nl || gLy >= nl) return;
    const double qs = -a.qscale * kInv2Pi;
    // D row m = 4 g + i of tile mt is target t = 16 mt + 4 g + i: ty = 2 mt + g / 2, tx = 4 (g & 1) + i
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        double *ur = pp.u + (size_t)(gLy * 8 + 2 * mt + (g >> 1)) * n + gLx * 8 + 4 * (g & 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) ur[i] = qs * acc[mt][i];
    }
    if (pp.M) {
        const int64_t ncell = (int64_t)nl * nl, cell = (int64_t)gLy * nl + gLx;
        double2 *Ml = pp.M + a.lv.off[a.L];
        // D rows 16 mt + 4 g + {0,1} and {2,3} are (Re, Im) of coefficients 8 mt + 2 g + {0, 1}
#pragma unroll
        for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int k = 8 * mt + 2 * g + j;
                if (k < P)
                    Ml[k * ncell + cell] = make_double2(a.qscale * (double)pm[mt][2 * j],
                                                        a.qscale * (double)pm[mt][2 * j + 1]);
            }
    }
}

// FP32 leaf stage with the near set of a MAC theta (radius K >= 2): the
// contraction of k_leaf_mfma32 over the leaf offsets of the lattice disk
// (rows |oy| <= K, columns |ox| <= kx(|oy|)) instead of the 3x3 block.
// Block = 8x8 target leaves, wave w = leaves 16w..16w+15 (rows 2w, 2w+1), as
// there.  LDS: the (8+2K)^2-leaf q tile in FP32 at
//   (pos/4) * TW*72 + row*72 + (pos%4)*16 + col,   col < TW = 8 + 2K <= 16,
// so one B read (8 columns x 2 rows x 4 positions) covers the 64 banks once;
// the kernel table T (side KS = 16K + 15) with rows KS floats apart, so that
// two blocks share a CU at K = 3 (80.4 KB).  An A read spans 2 rows x 11
// columns; with the row pitch 63 = -1 (mod 64) at K = 3 the two rows share 10
// banks, a 2-way conflict.  A conflict-free pitch (11..53 mod 64) needs at
// least 75 floats per row, which leaves one block per CU; measured at K = 3
// the conflicts cost 9.7e6 cycles per launch, LDS work in all 13% of the CU
// cycles while the matrix cores are busy 69% of them.  Bounds: row and
// column of a B read are ly + K + oy and lx + K + ox, both in [0, TW); a T
// index dy + 8K + 7 with |dy| <= 8K + 7 stays in [0, 16K + 15).
template <int P, int K>
__global__ __launch_bounds__(256) void k_leaf_wide_mfma32(LeafArgs a, const float *__restrict__ kt32,
                                                          const float *__restrict__ w32)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on) return;
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int TW = 8 + 2 * K, PS = TW * 72, KC = 8 * K + 7, KS = 2 * KC + 1, TS = KS;
    constexpr int MTP = (2 * P + 15) / 16;      // P2M row tiles
    static_assert(TW <= 16 && KS <= TS, "tile layout");
    __shared__ float sq[16 * PS];
    __shared__ float st[KS * TS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, nl = a.nl;
    const int TX0 = blockIdx.x * 8, TY0 = blockIdx.y * 8;
    const int X0 = (TX0 - K) * 8, Y0 = (TY0 - K) * 8;
    constexpr int PW = 8 * TW, NE = PW * PW, NB = 8, NT = (KS * KS + 255) / 256;
    // the kernel table's loads are all issued before the charge tile's, and
    // stored once those are in
    float w[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int e = tid + 256 * i;
        w[i] = e < KS * KS ? kt32[e] : 0.0f;
    }
#pragma unroll 1
    for (int base = 0; base < NE; base += 256 * NB) {
        float v[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = base + tid + 256 * i;
            const int yy = e / PW, xx = e - yy * PW;
            const int gx = X0 + xx, gy = Y0 + yy;
            v[i] = (e < NE && gx >= 0 && gx < n && gy >= 0 && gy < n) ? (float)pp.q[(size_t)gy * n + gx] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = base + tid + 256 * i;
            const int yy = e / PW, xx = e - yy * PW;
            const int pos = (yy & 7) * 8 + (xx & 7);
            if (e < NE) sq[(pos >> 2) * PS + (yy >> 3) * 72 + (pos & 3) * 16 + (xx >> 3)] = v[i];
        }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int e = tid + 256 * i;
        if (e < KS * KS) st[(e / KS) * TS + e % KS] = w[i];
    }
    __syncthreads();
    const int g = lane >> 4, m16 = lane & 15;
    const int lx = m16 & 7, ly = 2 * wave + (m16 >> 3);   // leaf of this lane's B column
    // A operand of lane: target t = 16 mt + m16 -> tx = lane & 7, ty = 2 mt + ((lane >> 3) & 1);
    // source s = 4 kk + g -> sx = 4 (kk & 1) + g, sy = kk >> 1
    const int abase = (KC - ((lane >> 3) & 1)) * TS + KC + g - (lane & 7);
    const int bbase = (ly + K) * 72 + g * 16 + lx + K;
    double acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mt][i] = 0.0;
#pragma unroll 1
    for (int oy = -K; oy <= K; ++oy) {
        const int kxo = near_kx(a.kxp, oy < 0 ? -oy : oy);
#pragma unroll 1
        for (int ox = -kxo; ox <= kxo; ++ox) {
            f4 c[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) c[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            const float *Ab = st + abase + 8 * oy * TS + 8 * ox;
            const float *Bb = sq + bbase + oy * 72 + ox;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const float b = Bb[kk * PS];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    c[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ab[((kk >> 1) - 2 * mt) * TS + 4 * (kk & 1)], b,
                                                                 c[mt], 0, 0, 0);
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[mt][i] += (double)c[mt][i];
        }
    }
    // P2M: rows of w32 against the centre leaves
    f4 pm[MTP];
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt) pm[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    if (pp.M) {
        const float *Bb = sq + bbase;
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const float b = Bb[kk * PS];
#pragma unroll
            for (int mt = 0; mt < MTP; ++mt)
                pm[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(w32[(16 * mt + m16) * 64 + 4 * kk + g], b,
                                                              pm[mt], 0, 0, 0);
        }
    }
    const int gLx = TX0 + lx, gLy = TY0 + ly;
    if (gLx >= nl || gLy >= nl) return;
    const double qs = -a.qscale * kInv2Pi;
    // D row m = 4 g + i of tile mt is target t = 16 mt + 4 g + i: ty = 2 mt + g / 2, tx = 4 (g & 1) + i
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        double *ur = pp.u + (size_t)(gLy * 8 + 2 * mt + (g >> 1)) * n + gLx * 8 + 4 * (g & 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) ur[i] = qs * acc[mt][i];
    }
    if (pp.M) {
        const int64_t ncell = (int64_t)nl * nl, cell = (int64_t)gLy * nl + gLx;
        double2 *Ml = pp.M + a.lv.off[a.L];
        // D rows 16 mt + 4 g + {0,1} and {2,3} are (Re, Im) of coefficients 8 mt + 2 g + {0, 1}
#pragma unroll
        for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int k = 8 * mt + 2 * g + j;
                if (k < P)
                    Ml[k * ncell + cell] = make_double2(a.qscale * (double)pm[mt][2 * j],
                                                        a.qscale * (double)pm[mt][2 * j + 1]);
            }
    }
}

// Split-precision variants of the leaf stage: the contraction of
// k_leaf_mfma32 on the 16-bit matrix cores (v_mfma_f32_16x16x32_f16 or
// _bf16, K = 32 source positions = four source rows per product).  Each
// operand is a pair x = hi + lo of 16-bit numbers: the kernel table T and
// the P2M weights were split at setup, the charges are scaled per block by
// a power of two (so that |q| <= 1 over the staged tile) and split here.
// FP16 pairs (11 significant bits each, about 2^-22 together) sum
// hi*hi + hi*lo + lo*hi; BF16 pairs (8 bits each, about 2^-16 together) also
// take lo*lo, which is as large as their representation error.  Products
// accumulate in FP32 and are folded into FP64 per leaf offset.  The A
// fragment of a lane is 8 consecutive entries of one T row starting at
// column 8 ox - tx + 15; T sits in LDS in 8 copies shifted by c = 7 - tx
// columns so that this start is 16-byte aligned, rows 20 dwords apart and
// copies 648 dwords apart (= 8 mod 64), which spreads a 16-lane read over
// distinct banks.  The q tile is [leaf row][leaf][pos] with 72 halves per
// leaf and 832 per leaf row (10 leaves and 112 halves of padding): a 16-lane
// B read covers two adjacent leaf rows of 8 leaves, and a row pitch of 416
// dwords (32 mod 64) puts the second row's 16-byte reads on the banks the
// first row's leave free.  MFMA lane layout (16x16x32, both types):
// A[l%16][8(l/16)+i], B[8(l/16)+i][l%16], D[4(l/16)+i][l%16].
constexpr int kT16Row = 40, kT16Copy = 31 * 40, kT16Pitch = 1296, kQ16Leaf = 72, kQ16RowP = 832;

typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename H> struct Split16;
template <> struct Split16<_Float16> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static constexpr bool kLoLo = false;
    // FP64 -> FP32 -> FP16, each rounded to nearest.  gfx950 has no FP64 ->
    // FP16 conversion, and the compiler turns a plain double-to-half cast
    // (even through a float) into the correctly rounded software sequence,
    // ~40 instructions per value and most of this kernel's VALU work.  A
    // multiply by `one` (1.0f, not known at compile time) keeps the two
    // steps apart: v_cvt_f32_f64 + v_fma_mixlo_f16.  The pair stays exact to
    // lo's rounding, since lo = x - hi is formed in FP64 whatever hi's last bit.
    __device__ static _Float16 cvt(double x, float one) { return (_Float16)((float)x * one); }
    __device__ static f4_t mfma(v8 a, v8 b, f4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Split16<__bf16> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static constexpr bool kLoLo = true;
    // the same two steps as Split16<_Float16>::cvt (a plain cast is again
    // folded into one FP64 -> BF16 rounding, done in software)
    __device__ static __bf16 cvt(double x, float one) { return (__bf16)((float)x * one); }
    __device__ static f4_t mfma(v8 a, v8 b, f4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// One block per CU-slot loops over the 8 x 8-leaf tiles t = blockIdx.x,
// blockIdx.x + gridDim.x, ... (ntx tiles per row, ntiles in all): the kernel
// table is staged once per block, and the next tile's charges are loaded
// into registers while the current tile's products run.  A thread holds row
// segments sg = tid + 256 i (i < 4, sg < 800) of the 80 x 80 q tile, 8
// consecutive nodes of one leaf row each, and writes each segment's halves
// as one 16-byte store.
template <int P, typename H>
__global__ __launch_bounds__(256) void k_leaf_mfma16(LeafArgs a, const H *__restrict__ kt16,
                                                     const H *__restrict__ w16, int ntx, int ntiles)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on || (int)blockIdx.x >= ntiles) return;
    using S = Split16<H>;
    typedef typename S::v8 h8;
    typedef f4_t f4;
    constexpr int MTP = (2 * P + 15) / 16;
    __shared__ __align__(16) H st[2][8 * kT16Pitch];
    __shared__ __align__(16) H sqh[10 * kQ16RowP], sql[10 * kQ16RowP];
    __shared__ double smax[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, nl = a.nl;
    // kernel table: 2 x 8 copies of 31 rows x 40 halves, contiguous in global
    // memory and copied in 16-byte units (unit e = halves 8e..8e+7, copy
    // e / 155), each copy padded to kT16Pitch halves in LDS.  A thread issues
    // all its table loads and the first tile's charge loads before it waits.
    constexpr int kTabUnits = 2 * 8 * kT16Copy / 8, kTabIt = (kTabUnits + 255) / 256;
    h8 tb[kTabIt];
#pragma unroll
    for (int i = 0; i < kTabIt; ++i) {
        const int e = tid + 256 * i;
        if (e < kTabUnits) tb[i] = *(const h8 *)&kt16[8 * e];
    }
    double v[4][8];
    auto load = [&](int t) {
        const int X0 = ((t % ntx) * 8 - 1) * 8, Y0 = ((t / ntx) * 8 - 1) * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int sg = tid + 256 * i, yy = sg / 10, gy = Y0 + yy;
            const int gx0 = X0 + 8 * (sg - yy * 10);
            const bool rowin = sg < 800 && gy >= 0 && gy < n;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int gx = gx0 + j;
                v[i][j] = (rowin && gx >= 0 && gx < n) ? pp.q[(size_t)gy * n + gx] : 0.0;
            }
        }
    };
    load(blockIdx.x);
    H *const stp = &st[0][0];
#pragma unroll
    for (int i = 0; i < kTabIt; ++i) {
        const int e = tid + 256 * i;
        if (e < kTabUnits) *(h8 *)&stp[8 * e + (kT16Pitch - kT16Copy) * (e / (kT16Copy / 8))] = tb[i];
    }
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int TX0 = (t % ntx) * 8, TY0 = (t / ntx) * 8;
        double mx = 0.0;
    #pragma unroll
        for (int i = 0; i < 4; ++i)
    #pragma unroll
            for (int j = 0; j < 8; ++j) mx = fmax(mx, fabs(v[i][j]));
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        if (lane == 0) smax[wave] = mx;
        // (the previous tile's reads of the q tile and of smax are done)
        __syncthreads();
        const double tmax = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
        int ex = 0;
        if (tmax > 0.0) (void)frexp(tmax, &ex);          // tmax < 2^ex
        ex = max(-100, min(100, ex));                     // (float) of both scales stays exact
        const double scale = ldexp(1.0, -ex), iscale = ldexp(1.0, ex);
        const float one = (float)scale * (float)iscale;   // 1.0f, a run-time value (see Split16)
    #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int sg = tid + 256 * i;
            if (sg < 800) {
                const int yy = sg / 10, jx = sg - yy * 10;
                const int at = (yy >> 3) * kQ16RowP + jx * kQ16Leaf + (yy & 7) * 8;
                h8 vh, vl;
    #pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const double x = v[i][j] * scale;
                    const H hi = S::cvt(x, one);
                    vh[j] = hi;
                    vl[j] = S::cvt(x - (double)(float)hi, one);
                }
                *(h8 *)&sqh[at] = vh;
                *(h8 *)&sql[at] = vl;
            }
        }
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) load(t + gridDim.x);
        const int g = lane >> 4, m16 = lane & 15;
        const int nloc = 16 * wave + m16;
        const int lx = nloc & 7, ly = nloc >> 3;
        // A: target t = 16 mt + m16 (tx = lane & 7, ty = 2 mt + ((lane >> 3) & 1)),
        //    source rows sy = 4 ks + g, columns from 8 ox - tx + 15 in copy 7 - tx
        const int tx = lane & 7, tyb = (lane >> 3) & 1;
        const int abase = (7 - tx) * kT16Pitch + (15 - tyb + g) * kT16Row + 8;
        const int bbase = (ly + 1) * kQ16RowP + (lx + 1) * kQ16Leaf + 8 * g;
        double acc[4][4];
    #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
    #pragma unroll
            for (int i = 0; i < 4; ++i) acc[mt][i] = 0.0;
        // leaf offsets column by column (ox), rows oy = -1, 0, 1 within: the A
        // fragment of (oy, ks, mt) is T row shift 8 oy + 4 ks - 2 mt, so one
        // offset row takes 6 distinct fragments and the next row shares 2 of
        // them, which stay in registers (fh, fl: shifts 8 oy - 6 .. 8 oy + 4)
    #pragma unroll 1
        for (int ox = -1; ox <= 1; ++ox) {
            h8 fh[6], fl[6];
            const int acol = abase + 8 * ox;
    #pragma unroll
            for (int f = 0; f < 6; ++f) {
                fh[f] = *(const h8 *)&st[0][acol + (2 * f - 14) * kT16Row];
                fl[f] = *(const h8 *)&st[1][acol + (2 * f - 14) * kT16Row];
            }
    #pragma unroll
            for (int oyi = 0; oyi < 3; ++oyi) {
                const int oy = oyi - 1;
                if (oyi > 0) {
    #pragma unroll
                    for (int f = 0; f < 2; ++f) {
                        fh[f] = fh[f + 4];
                        fl[f] = fl[f + 4];
                    }
    #pragma unroll
                    for (int f = 2; f < 6; ++f) {
                        const int ai = acol + (8 * oy + 2 * f - 6) * kT16Row;
                        fh[f] = *(const h8 *)&st[0][ai];
                        fl[f] = *(const h8 *)&st[1][ai];
                    }
                }
                f4 c[4];
    #pragma unroll
                for (int mt = 0; mt < 4; ++mt) c[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
                const int boff = bbase + oy * kQ16RowP + ox * kQ16Leaf;
    #pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const h8 bh = *(const h8 *)&sqh[boff + 32 * ks];
                    const h8 bl = *(const h8 *)&sql[boff + 32 * ks];
    #pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        const h8 ah = fh[2 * ks - mt + 3], al = fl[2 * ks - mt + 3];
                        if constexpr (S::kLoLo) c[mt] = S::mfma(al, bl, c[mt]);
                        c[mt] = S::mfma(ah, bl, c[mt]);
                        c[mt] = S::mfma(al, bh, c[mt]);
                        c[mt] = S::mfma(ah, bh, c[mt]);
                    }
                }
    #pragma unroll
                for (int mt = 0; mt < 4; ++mt)
    #pragma unroll
                    for (int i = 0; i < 4; ++i) acc[mt][i] += (double)c[mt][i];
            }
        }
        f4 pm[MTP];
    #pragma unroll
        for (int mt = 0; mt < MTP; ++mt) pm[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        if (pp.M) {
    #pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const h8 bh = *(const h8 *)&sqh[bbase + 32 * ks];
                const h8 bl = *(const h8 *)&sql[bbase + 32 * ks];
    #pragma unroll
                for (int mt = 0; mt < MTP; ++mt) {
                    const size_t wi = (size_t)(16 * mt + m16) * 64 + 32 * ks + 8 * g;
                    const h8 wh = *(const h8 *)&w16[wi];
                    const h8 wl = *(const h8 *)&w16[(size_t)16 * MTP * 64 + wi];
                    if constexpr (S::kLoLo) pm[mt] = S::mfma(wl, bl, pm[mt]);
                    pm[mt] = S::mfma(wh, bl, pm[mt]);
                    pm[mt] = S::mfma(wl, bh, pm[mt]);
                    pm[mt] = S::mfma(wh, bh, pm[mt]);
                }
            }
        }
        const int gLx = TX0 + lx, gLy = TY0 + ly;
        if (gLx < nl && gLy < nl) {
            const double qs = -a.qscale * iscale * kInv2Pi;
    #pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                double *ur = pp.u + (size_t)(gLy * 8 + 2 * mt + (g >> 1)) * n + gLx * 8 + 4 * (g & 1);
    #pragma unroll
                for (int i = 0; i < 4; ++i) ur[i] = qs * acc[mt][i];
            }
            if (pp.M) {
                const int64_t ncell = (int64_t)nl * nl, cell = (int64_t)gLy * nl + gLx;
                double2 *Ml = pp.M + a.lv.off[a.L];
                const double ms = a.qscale * iscale;
    #pragma unroll
                for (int mt = 0; mt < MTP; ++mt)
    #pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int k = 8 * mt + 2 * g + j;
                        if (k < P)
                            Ml[k * ncell + cell] = make_double2(ms * (double)pm[mt][2 * j],
                                                                ms * (double)pm[mt][2 * j + 1]);
                    }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// M2L of the split 16-bit plans on the matrix cores (Sec. 5.3 item 3 as a
// dense contraction).  Per list entry e of a parity class, the translation is
// the real 2P x 2P matrix T_e of  L~_n = sum_k a_n H_{n+k} b_k M~_k  (rows
// 2n + {Re, Im}, columns 2k + {Re, Im}; the level's log w term of H_0 is
// added apart, in FP64), built and split into 16-bit pairs at setup, padded
// to MP rows and KP columns.  For the 64 same-parity target cells of a class
// (columns) the block computes
//   D = sum_e T_e S_e,   S_e = the source multipoles at target + offset_e,
// with the list entries concatenated along K, so that only the rows pad:
// K step t takes groups 4t..4t+3 of KP/8 = G groups of 8 columns per entry,
// lane group g = l/16 the group 4t + g (one entry and 8 columns of it).
// v_mfma_f32_16x16x32_{f16,bf16}: A[l%16][8(l/16)+i], B[8(l/16)+i][l%16],
// D[4(l/16)+i][l%16].  Operands are pairs x = hi + lo; the sources are
// scaled per tile by a power of two (|M~| <= 1 on the staged tile) and split
// here; hi*hi + hi*lo + lo*hi products (BF16 also lo*lo) accumulate in FP32.
// Block layout as k_m2l: a 16x16 target tile and share item.part of nsplit
// of the lists, 12 waves = 4 parity classes x 3 thirds of the share, the
// thirds summed in LDS in a fixed order.  LDS: the tile's sources as [cell]
// [KP] hi and lo halves, then M~_0 of every cell in FP64 (for the log w term).
// Six waves per SIMD (at most 80 VGPRs) let two 12-wave blocks share a CU.
// ---------------------------------------------------------------------------
// largest share of one class's list a k_m2l_mfma16 block takes (the list
// rule's 27 entries at split 1)
constexpr int kM2L16MaxShare = 32;

// dynamic LDS of k_m2l_mfma16 for source tiles of side rw: the staged
// hi/lo halves and M~_0, or the reduction of the thirds, whichever is larger
template <int P>
constexpr size_t m2l16_lds(int rw)
{
    constexpr int KP = 8 * ((2 * P + 7) / 8), MT = (2 * P + 15) / 16;
    const size_t stage = (size_t)rw * rw * (KP * 2 * 2 + 16);
    const size_t red = (size_t)4 * 64 * 16 * MT * sizeof(float);
    return stage > red ? stage : red;
}

template <int P, typename H>
__global__ __launch_bounds__(768, P <= 12 ? 6 : 1) void k_m2l_mfma16(const M2LItem *__restrict__ items,
                                                    const double2 *__restrict__ M,
                                                    double2 *__restrict__ Lm, int64_t lm_part,
                                                    int nsplit, LevelInfo lv,
                                                    const H *__restrict__ T,
                                                    const int4 *__restrict__ offs, int nlist,
                                                    int halo, RhsSet rh)
{
    using S = Split16<H>;
    typedef typename S::v8 h8;
    typedef f4_t f4;
    constexpr int KP = 8 * ((2 * P + 7) / 8), MP = 16 * ((2 * P + 15) / 16);
    constexpr int MT = MP / 16, G = KP / 8;
    if (!rhs_active(rh, blockIdx.z)) return;
    M += blockIdx.z * rh.se;
    Lm += blockIdx.z * rh.se;
    extern __shared__ __align__(16) unsigned char sm_raw[];
    __shared__ double smax[12];
    __shared__ int sdel[4 * kM2L16MaxShare];   // source-cell offset in the tile of each entry of the share
    const M2LItem it = items[blockIdx.x];
    const int l = it.level, nc = 1 << l;
    const int tw = nc < 16 ? nc : 16;
    const int RW = tw + 2 * halo, RR = RW * RW;
    const int64_t ncell = (int64_t)nc * nc;
    H *sh = reinterpret_cast<H *>(sm_raw);                       // [RR][KP] hi
    H *sl = sh + (size_t)RR * KP;                                // [RR][KP] lo
    double2 *s0 = reinterpret_cast<double2 *>(sl + (size_t)RR * KP);   // [RR] M~_0
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double2 *Ml = M + lv.off[l];
    // the block's share of each class's list: entries [lo, lo + cnt)
    const int per = (nlist + nsplit - 1) / nsplit;
    const int lo = it.part * per, cnt = max(0, min(per, nlist - lo));
    if (tid < 4 * cnt) {
        const int w = tid / cnt, e = tid - w * cnt;
        const int4 od = offs[w * nlist + lo + e];
        sdel[w * kM2L16MaxShare + e] = od.y * RW + od.x;
    }
    // stage: thread r < RR holds the P coefficients of tile cell r
    double2 v[P];
    double mx = 0.0;
    const bool has = tid < RR;
    {
        const int sy = has ? tid / RW : 0, sx = has ? tid - sy * RW : 0;
        const int gx = it.tx0 - halo + sx, gy = it.ty0 - halo + sy;
        const bool in = has && gx >= 0 && gx < nc && gy >= 0 && gy < nc;
        const int64_t gi = in ? (int64_t)gy * nc + gx : 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            v[k] = in ? Ml[k * ncell + gi] : make_double2(0.0, 0.0);
            mx = fmax(mx, fmax(fabs(v[k].x), fabs(v[k].y)));
        }
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) smax[wave] = mx;
    __syncthreads();
    double tmax = 0.0;
#pragma unroll
    for (int w = 0; w < 12; ++w) tmax = fmax(tmax, smax[w]);
    int ex = 0;
    if (tmax > 0.0) (void)frexp(tmax, &ex);
    ex = max(-100, min(100, ex));
    const double scale = ldexp(1.0, -ex), iscale = ldexp(1.0, ex);
    const float one = (float)scale * (float)iscale;   // 1.0f, a run-time value (see Split16)
    if (has) {
        // the cell's 2P values (Re, Im of each coefficient, zero padded to KP)
        // as pairs, written 8 halves at a time
#pragma unroll
        for (int q = 0; q < G; ++q) {
            h8 vh, vl;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int kk = 8 * q + i;
                const double x = kk < 2 * P ? ((kk & 1) ? v[kk >> 1].y : v[kk >> 1].x) * scale : 0.0;
                const H hx = S::cvt(x, one);
                vh[i] = hx;
                vl[i] = S::cvt(x - (double)(float)hx, one);
            }
            *(h8 *)&sh[tid * KP + 8 * q] = vh;
            *(h8 *)&sl[tid * KP + 8 * q] = vl;
        }
        s0[tid] = v[0];
    }
    __syncthreads();
    const int cls = wave & 3, grp = wave >> 2;
    const int px = cls & 1, py = cls >> 1;
    const int col = lane & 15, g = lane >> 4;
    // the four target cells of this lane (one per 16-column tile j) and the
    // base of their source cells in the staged tile
    int cbase[4];
    bool act[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = 16 * j + col;
        const int ltx = 2 * (c & 7) + px, lty = 2 * (c >> 3) + py;
        act[j] = ltx < tw && lty < tw;
        cbase[j] = (lty + halo) * RW + ltx + halo;
    }
    // this wave's entries: third grp of the block's share of the list
    const int chunk = (cnt + 2) / 3;
    const int e0 = lo + grp * chunk;
    const int nown = max(0, min(chunk, cnt - grp * chunk));
    const int ngroups = nown * G, nsteps = (ngroups + 3) / 4;
    const int *dl = sdel + cls * kM2L16MaxShare;   // dl[e - lo], e in [lo, lo + cnt)
    const size_t lo_half = (size_t)4 * nlist * MP * KP;   // the lo parts follow the hi parts
    f4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[mt][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int t = 0; t < nsteps; ++t) {
        const int gi = 4 * t + g;
        const bool valid = gi < ngroups;
        const int e = e0 + (valid ? gi / G : 0), q = valid ? gi % G : 0;
        const int sd = dl[e - lo];
        h8 ah[MT], al[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const size_t ai = ((size_t)(cls * nlist + e) * MP + 16 * mt + col) * KP + 8 * q;
            ah[mt] = *(const h8 *)&T[ai];
            al[mt] = *(const h8 *)&T[lo_half + ai];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            h8 bh, bl;
            if (valid && act[j]) {
                const int si = (cbase[j] + sd) * KP + 8 * q;
                bh = *(const h8 *)&sh[si];
                bl = *(const h8 *)&sl[si];
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bh[i] = S::cvt(0.0, one);
                    bl[i] = S::cvt(0.0, one);
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                if constexpr (S::kLoLo) acc[mt][j] = S::mfma(al[mt], bl, acc[mt][j]);
                acc[mt][j] = S::mfma(ah[mt], bl, acc[mt][j]);
                acc[mt][j] = S::mfma(al[mt], bh, acc[mt][j]);
                acc[mt][j] = S::mfma(ah[mt], bh, acc[mt][j]);
            }
        }
    }
    // the log w term of H_0 adds log w * sum_e M~_0(source) to L~_0 (D rows
    // 0, 1: lanes of group 0), each wave over its own entries, summed in FP64
    // and added to the FP32 accumulators at the tile's scale before the
    // thirds are summed (and before that sum reuses the LDS)
    if (g == 0) {
        const double lws = lv.logw[l] * scale;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double cx = 0.0, cy = 0.0;
#pragma unroll
            for (int ee = 0; ee < (kM2L16MaxShare + 2) / 3; ++ee)
                if (ee < nown && act[j]) {
                    const double2 m0 = s0[cbase[j] + dl[e0 + ee - lo]];
                    cx += m0.x;
                    cy += m0.y;
                }
            acc[0][j][0] += (float)(lws * cx);
            acc[0][j][1] += (float)(lws * cy);
        }
    }
    // sum the three thirds: (third 0 + third 1) + third 2, through the
    // source region of LDS, component-major ([16 MT][4 classes x 64 lanes]
    // floats, so that a wave's 64 lanes write 64 consecutive words)
    float *red = reinterpret_cast<float *>(sm_raw);
    const int slot = cls * 64 + lane;
    for (int gg = 1; gg < 3; ++gg) {
        __syncthreads();
        if (grp == gg) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) red[((mt * 4 + j) * 4 + i) * 256 + slot] = acc[mt][j][i];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[mt][j][i] += red[((mt * 4 + j) * 4 + i) * 256 + slot];
        }
    }
    if (grp != 0) return;
    // rows 16 mt + 4 g + i of D: coefficient n = row / 2, (Re, Im) = row & 1
    double2 *out = Lm + it.part * lm_part + lv.off[l];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!act[j]) continue;
        const int c = 16 * j + col;
        const int tx = it.tx0 + 2 * (c & 7) + px, ty = it.ty0 + 2 * (c >> 3) + py;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; i += 2) {
                const int row = 16 * mt + 4 * g + i, n = row >> 1;
                if (n >= P) continue;
                out[n * ncell + (int64_t)ty * nc + tx] =
                    make_double2(iscale * (double)acc[mt][j][i], iscale * (double)acc[mt][j][i + 1]);
            }
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

// Re sum_k L_k tau^k
template <int P>
__device__ __forceinline__ double l2p_eval(const double2 *__restrict__ Lc, double2 tau)
{
    double s = 0.0;
    double2 pw = make_double2(1.0, 0.0);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double2 c = Lc[k];
        s = fma(c.x, pw.x, fma(-c.y, pw.y, s));
        pw = cmul(pw, tau);
    }
    return s;
}

// ---------------------------------------------------------------------------
// Pass-1 potential at the ring nodes and the right-hand side of the boundary
// solve.  A block of 8 waves takes the eight nodes (side s, k) and
// (s, n-1-k), s = 0..3, of one k < n/2, one node per wave.  Each node's near
// field comes from the in-domain leaves of the near set around its boundary
// leaf (at most 6 of the 3x3 block with the list rule), split over the lanes
// and summed with shuffles; its far field is the L2P of that leaf's local
// expansion.  Then phi and, with bh, b = -phi as the DFT over the sides
// (b^_0 = sum_s b_s, b^_2 = sum_s (-1)^s b_s, b^_1 = sum_s i^(-s) b_s) split
// into even and odd parts b^[k] +- b^[n-1-k], the layout the boundary
// solve's products read: bh = [mode 0: even | odd][mode 2: even | odd]
// [mode 1: even | odd].
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(512) void k_ring_targets(LeafArgs a, double *__restrict__ phi,
                                                      double2 *__restrict__ bh)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on) return;
    phi += blockIdx.z * a.rh.sr;
    if (bh) bh += blockIdx.z * a.rh.sb;
    __shared__ double val[8];
    const int kq = blockIdx.x, v = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.n, nl = a.nl, m = n >> 1;
    const int t = (v & 3) * n + (v < 4 ? kq : n - 1 - kq);
    int Ix, Iy;
    ring_node(t, n, Ix, Iy);
    const int lx = leaf_of(Ix, nl), ly = leaf_of(Iy, nl);
    double near = 0.0;
    const int ia = lane & 7, jb = lane >> 3;
    for (int b = -a.K; b <= a.K; ++b) {
        const int kb = near_kx(a.kxp, b < 0 ? -b : b);
        for (int c = -kb; c <= kb; ++c) {
            const int qx = lx + c, qy = ly + b;
            if (qx < 0 || qy < 0 || qx >= nl || qy >= nl) continue;
            const int gx = qx * 8 + ia, gy = qy * 8 + jb;
            const int dx = abs(Ix - (gx + 1)), dy = abs(Iy - (gy + 1));
            near = fma(pp.q[(size_t)gy * n + gx], a.rtab[dy * a.rs + dx], near);
        }
    }
    near = wave_sum(near);
    if (lane == 0) {
        double far = 0.0;
        if (a.far) {
            const int64_t ncell = (int64_t)nl * nl, cell = (int64_t)ly * nl + lx;
            const double2 *Ll = pp.Lt + a.lv.off[a.L];
            double2 Lc[P];
#pragma unroll
            for (int k = 0; k < P; ++k) Lc[k] = Ll[k * ncell + cell];
            far = l2p_eval<P>(Lc, make_double2((Ix - 8 * lx - 4.5) * 0.125, (Iy - 8 * ly - 4.5) * 0.125));
        }
        const double ph = -(fma(a.qscale, near, far)) * kInv2Pi;
        phi[t] = ph;
        val[v] = ph;
    }
    __syncthreads();
    if (!bh || threadIdx.x != 0) return;
    const double b0 = -val[0], b1 = -val[1], b2 = -val[2], b3 = -val[3];
    const double c0 = -val[4], c1 = -val[5], c2 = -val[6], c3 = -val[7];
    const double m0 = (b0 + b1) + (b2 + b3), n0 = (c0 + c1) + (c2 + c3);
    const double m2 = (b0 - b1) + (b2 - b3), n2 = (c0 - c1) + (c2 - c3);
    const double2 m1 = make_double2(b0 - b2, b3 - b1), n1 = make_double2(c0 - c2, c3 - c1);
    bh[kq] = make_double2(m0 + n0, 0.0);
    bh[m + kq] = make_double2(m0 - n0, 0.0);
    bh[n + kq] = make_double2(m2 + n2, 0.0);
    bh[n + m + kq] = make_double2(m2 - n2, 0.0);
    bh[2 * n + kq] = make_double2(m1.x + n1.x, m1.y + n1.y);
    bh[2 * n + m + kq] = make_double2(m1.x - n1.x, m1.y - n1.y);
}

// lattice coordinates of node k of side s
__device__ __forceinline__ void side_node(int s, int k, int n, int &Ix, int &Iy)
{
    if (s == 0) { Ix = k + 1; Iy = 0; }
    else if (s == 1) { Ix = n + 1; Iy = k + 1; }
    else if (s == 2) { Ix = n - k; Iy = n + 1; }
    else { Ix = 0; Iy = n - k; }
}

// Pass 2 upward, all levels at once: the multipoles of the ring charges in
// every boundary cell of levels 2..L by direct P2M from the ring nodes the
// cell borders (M~_0 = sum c, M~_k = -sum c tau^k / k, tau = node offset
// from the cell centre in cell widths; Sec. 5.3 item 1).  On p-term
// expansions this equals P2M at the leaves followed by M2M up the tree (a
// parent's first p coefficients depend only on its children's first p),
// without a chain of dependent levels.  One wave per boundary cell, items
// (level, ix, iy); the lanes split the cell's s = n / 2^l nodes per side and
// the wave sums them with shuffles.  The charges h sigma are formed here from
// the boundary solve's products (ring_sigma); the leaf-level waves, which
// see every node exactly once, also store them (rq, and sigma to sig_out).
template <int P>
__global__ __launch_bounds__(256) void k_p2m_ring(const int4 *__restrict__ cells, int ncells,
                                                  const double2 *__restrict__ sh, double h,
                                                  double *__restrict__ rq,
                                                  double *__restrict__ sig_out,
                                                  double2 *__restrict__ M, LevelInfo lv, int n,
                                                  int L, RhsSet rh)
{
    if (!rhs_active(rh, blockIdx.z)) return;
    sh += blockIdx.z * rh.sb;
    rq += blockIdx.z * rh.sr;
    if (sig_out) sig_out += blockIdx.z * rh.sr;
    M += blockIdx.z * rh.se;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= ncells) return;
    const int4 it = cells[w];
    const int l = it.x, ix = it.y, iy = it.z, nc = 1 << l, s = n >> l;
    int sd[2], k0[2], r = 0;
    if (iy == 0) { sd[r] = 0; k0[r] = s * ix; ++r; }
    if (ix == nc - 1 && r < 2) { sd[r] = 1; k0[r] = s * iy; ++r; }
    if (iy == nc - 1 && r < 2) { sd[r] = 2; k0[r] = n - s * ix - s; ++r; }
    if (ix == 0 && r < 2) { sd[r] = 3; k0[r] = n - s * iy - s; ++r; }
    const double inv = 1.0 / (double)s;
    const double cx = s * ix + 0.5 * s + 0.5, cy = s * iy + 0.5 * s + 0.5;
    double2 m[P];
#pragma unroll
    for (int k = 0; k < P; ++k) m[k] = make_double2(0.0, 0.0);
    for (int q = 0; q < r; ++q)
        for (int j = lane; j < s; j += 64) {
            int Ix, Iy;
            side_node(sd[q], k0[q] + j, n, Ix, Iy);
            const double sg = ring_sigma(sh, sd[q], k0[q] + j, n);
            const double cq = h * sg;
            if (l == L) {
                rq[sd[q] * n + k0[q] + j] = cq;
                if (sig_out) sig_out[sd[q] * n + k0[q] + j] = sg;
            }
            const double2 tau = make_double2((Ix - cx) * inv, (Iy - cy) * inv);
            double2 pw = make_double2(1.0, 0.0);
            m[0].x += cq;
#pragma unroll
            for (int k = 1; k < P; ++k) {
                pw = cmul(pw, tau);
                m[k].x = fma(cq, pw.x, m[k].x);
                m[k].y = fma(cq, pw.y, m[k].y);
            }
        }
#pragma unroll
    for (int k = 0; k < P; ++k)
        for (int o = 32; o > 0; o >>= 1) {
            m[k].x += __shfl_xor(m[k].x, o);
            m[k].y += __shfl_xor(m[k].y, o);
        }
    if (lane != 0) return;
    const int64_t ncell = (int64_t)nc * nc, cell = (int64_t)iy * nc + ix;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double f = k == 0 ? 1.0 : -1.0 / (double)k;
        M[lv.off[l] + k * ncell + cell] = make_double2(f * m[k].x, f * m[k].y);
    }
}

// Pass 2 M2L: the multipoles are non-zero only in the boundary cells of each
// level, and those are in the interaction lists of cells at most 2K + 1 cells
// from the boundary (three with the list rule).  A wave takes one row of that band along one side
// (item = level, side, depth d, first coordinate along the side; lanes step
// by two, so all lanes share a parity class and hence one list).  For each
// list entry the source's boundary test is uniform except at the ends of
// the strip, and the Hankel generators are wave-uniform.  Bottom and top
// strips span the full width; left and right strips skip the rows the
// bottom and top strips own; levels with at most 8 cells per side are one
// "bottom" strip per row.  A block takes one item; its four waves split the
// list.
template <int P>
__global__ __launch_bounds__(256) void k_m2l_ring(const int4 *__restrict__ items, int nitems,
                                                  const double2 *__restrict__ M,
                                                  double2 *__restrict__ Lm, LevelInfo lv,
                                                  const double2 *__restrict__ hank,
                                                  const int4 *__restrict__ offs,
                                                  const double *__restrict__ a_n,
                                                  const double *__restrict__ b_k, int nlist,
                                                  RhsSet rh)
{
    // one item per block; wave w takes list entries w, w+4, ... and the four
    // partial sums are added in LDS in a fixed order
    __shared__ double2 red[3][P][64];
    if (!rhs_active(rh, blockIdx.z)) return;
    M += blockIdx.z * rh.se;
    Lm += blockIdx.z * rh.se;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int4 it = items[blockIdx.x];   // (level, side | depth << 2, start, end)
    const int l = it.x, side = it.y & 3, d = it.y >> 2, nc = 1 << l;
    const int a = it.z + 2 * lane;
    const bool valid = a < it.w;
    int ix, iy;
    if (side == 0) { ix = a; iy = d; }
    else if (side == 1) { ix = nc - 1 - d; iy = a; }
    else if (side == 2) { ix = a; iy = nc - 1 - d; }
    else { ix = d; iy = a; }
    const int64_t ncell = (int64_t)nc * nc;
    const double2 *Ml = M + lv.off[l];
    const int cls = __builtin_amdgcn_readfirstlane(((iy & 1) * 2 + (ix & 1)));
    const int4 *ol = offs + cls * nlist;
    const double logw = lv.logw[l];
    double2 acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int o = w; o < nlist; o += 4) {
        const int4 od = ol[o];
        const int sx = ix + od.x, sy = iy + od.y;
        const bool use = valid && sx >= 0 && sy >= 0 && sx < nc && sy < nc &&
                         (sx == 0 || sy == 0 || sx == nc - 1 || sy == nc - 1);
        if (!use) continue;
        const int64_t sc = (int64_t)sy * nc + sx;
        double2 m[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double2 v = Ml[k * ncell + sc];
            const double bk = b_k[k];
            m[k] = make_double2(v.x * bk, v.y * bk);
        }
        const double2 *H = hank + od.z * (2 * P - 1);
#pragma unroll
        for (int ss = 0; ss < 2 * P - 1; ++ss) {
            double2 h = H[ss];
            if (ss == 0) h.x -= logw;
#pragma unroll
            for (int nn = (ss < P ? 0 : ss - P + 1); nn <= (ss < P ? ss : P - 1); ++nn)
                cmac(acc[nn], h, m[ss - nn]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int k = 0; k < P; ++k) red[w - 1][k][lane] = acc[k];
    }
    __syncthreads();
    if (w != 0 || !valid) return;
    double2 *out = Lm + lv.off[l];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double2 b1 = red[0][k][lane], b2 = red[1][k][lane], b3 = red[2][k][lane];
        const double an = a_n[k];
        const double sx_ = ((acc[k].x + b1.x) + b2.x) + b3.x, sy_ = ((acc[k].y + b1.y) + b2.y) + b3.y;
        out[k * ncell + (int64_t)iy * nc + ix] = make_double2(an * sx_, an * sy_);
    }
}

// Pass 2 near field: u += -(1/2pi) sum over the ring nodes attached to the
// leaves of the near set around the target's leaf.  Ring node k of a side
// attaches to the boundary leaf it borders, so for each side the sum is a
// window of consecutive nodes (the near leaves along that side: three, 24
// nodes, with the list rule) with a kernel value from the lattice table, and
// only targets within K + 1 leaves of a side see it.
__device__ __forceinline__ double side_window(const double *__restrict__ rqs,
                                              const double *__restrict__ trow, int k0, int k1,
                                              int c, int sgn)
{
    // sum_{k0 <= k < k1} rqs[k] * trow[|c - sgn k|]
    double acc = 0.0;
#pragma unroll 8
    for (int k = k0; k < k1; ++k) acc = fma(rqs[k], trow[abs(c - sgn * k)], acc);
    return acc;
}

// the pass-2 near sum (before the -1/2pi) at grid point (gx, gy)
__device__ __forceinline__ double pass2_near_at(int gx, int gy, const double *__restrict__ rq,
                                                const double *__restrict__ rtab, int n, int nl,
                                                int K, int kxp, int rs)
{
    const int lx = gx >> 3, ly = gy >> 3;
    // lattice range [a, b) along a side covered by the near leaves l-k..l+k,
    // k = kx(distance of the target's leaf from that side)
    auto lo = [&](int l, int k) { return 8 * max(l - k, 0); };
    auto hi = [&](int l, int k) { return 8 * min(l + k, nl - 1) + 8; };
    double near = 0.0;
    const int db = ly, dr = nl - 1 - lx, dt = nl - 1 - ly, dl = lx;
    if (db <= K) {      // bottom: node k at (k+1, 0)
        const int k = near_kx(kxp, db);
        if (k >= 0) near += side_window(rq, rtab + (gy + 1) * rs, lo(lx, k), hi(lx, k), gx, 1);
    }
    if (dr <= K) {      // right: node k at (n+1, k+1)
        const int k = near_kx(kxp, dr);
        if (k >= 0) near += side_window(rq + n, rtab + (n - gx) * rs, lo(ly, k), hi(ly, k), gy, 1);
    }
    if (dt <= K) {      // top: node k at (n-k, n+1); Ix-1 = n-1-k in [ax, bx)
        const int k = near_kx(kxp, dt);
        if (k >= 0)
            near += side_window(rq + 2 * n, rtab + (n - gy) * rs, n - hi(lx, k), n - lo(lx, k),
                                gx - n + 1, -1);
    }
    if (dl <= K) {      // left: node k at (0, n-k); Iy-1 = n-1-k in [ay, by)
        const int k = near_kx(kxp, dl);
        if (k >= 0)
            near += side_window(rq + 3 * n, rtab + (gx + 1) * rs, n - hi(ly, k), n - lo(ly, k),
                                gy - n + 1, -1);
    }
    return near;
}

// Far field at every grid point, the last stage of an application:
//   u += -(1/2pi) Re sum_k (L~ring_k + L~vol_k) tau^k   (L2P, Sec. 5.3)
// over the leaves of an 8x8 tile.  The boundary-source expansions L~ring
// come from one of: none (a.Lt null), the leaf level of a.Lt, or (chain)
// the three levels below level L-3 built in LDS from the M2L sums Lm, with
// the level-(L-3) root read from a.Lt (chain 1) or built from its ancestors'
// M2L sums (chain 2, L - 3 <= 5).
// The volume expansions Lvol (leaf level), when given, are added in LDS, so
// the preconditioner's two passes share one sweep over u.
template <int P>
__global__ __launch_bounds__(256) void k_far_l2p(LeafArgs a, const double2 *__restrict__ Lm,
                                                 const double2 *__restrict__ B, int chain,
                                                 const double2 *__restrict__ Lvol)
{
    const LeafPtrs pp = rhs_ptrs(a);
    if (!pp.on) return;
    if (Lm) Lm += blockIdx.z * a.rh.se;
    if (Lvol) Lvol += blockIdx.z * a.rh.se;
    __shared__ double2 sB[4 * P * P];
    __shared__ double2 sm2l[P * 84];
    __shared__ double2 buf0[P * 64], buf1[P * 64];
    __shared__ double2 sanc[(kMaxAncestorLevel - 1) * P];
    const int n = a.n, nl = a.nl, tw = nl < 8 ? nl : 8, pw = tw * 8;
    const int lx0 = blockIdx.x * tw, ly0 = blockIdx.y * tw, cnt = tw * tw;
    const int ltw = __builtin_ctz(tw);
    const int64_t ncell = (int64_t)nl * nl;
    // coefficient k of tile leaf c = t & (cnt - 1), k = t / cnt, at the leaf level
    auto leaf_coef = [&](const double2 *__restrict__ base, int t) {
        const int k = t >> (2 * ltw), c = t & (cnt - 1);
        return base[a.lv.off[a.L] + k * ncell + (int64_t)(ly0 + (c >> ltw)) * nl + lx0 +
                    (c & (tw - 1))];
    };
    double2 vv[rounds256(P * 64)];
    if (Lvol) fetch(vv, P * cnt, [&](int t) { return leaf_coef(Lvol, t); });
    double2 *sL;
    if (chain) {
        const int r = a.L - 3, nr = 1 << r;
        const double2 *top =
            chain == 2 ? nullptr : pp.Lt + a.lv.off[r] + (int64_t)blockIdx.y * nr + blockIdx.x;
        sL = down_levels<P>(Lm, 1, 0, nullptr, B, a.lv, r, 3, blockIdx.x, blockIdx.y, sB, sm2l,
                            buf0, buf1, top, (int64_t)nr * nr, false, nullptr, sanc);
        if (Lvol) {
            put(vv, P * cnt, [&](int t, double2 x) {
                sL[t].x += x.x;
                sL[t].y += x.y;
            });
            __syncthreads();
        }
    } else {
        constexpr int R = rounds256(P * 64);
        double2 v[R];
        if (pp.Lt) fetch(v, P * cnt, [&](int t) { return leaf_coef(pp.Lt, t); });
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = threadIdx.x + 256 * r;
            if (t < P * cnt) {
                double2 y = pp.Lt ? v[r] : make_double2(0.0, 0.0);
                if (Lvol) {
                    y.x += vv[r].x;
                    y.y += vv[r].y;
                }
                buf0[t] = y;
            }
        }
        __syncthreads();
        sL = buf0;
    }
    if (pw == 64) {
        // element e = threadIdx.x + 256 r: column xx = threadIdx.x % 64 is fixed and row yy =
        // threadIdx.x / 64 + 4 r takes two in-leaf offsets (r even, r odd), so each class
        // of eight points shares the powers of tau (same per-point order of operations)
        const int xx = threadIdx.x & 63, y0 = threadIdx.x >> 6;
#pragma unroll
        for (int cls = 0; cls < 2; ++cls) {
            const double2 tau = make_double2(((xx & 7) - 3.5) * 0.125, (((y0 + 4 * cls) & 7) - 3.5) * 0.125);
            double far[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) far[j] = 0.0;
            double2 pk = make_double2(1.0, 0.0);
#pragma unroll
            for (int k = 0; k < P; ++k) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int yy = y0 + 4 * (2 * j + cls);
                    const double2 c = sL[k * 64 + (yy >> 3) * 8 + (xx >> 3)];
                    far[j] = fma(c.x, pk.x, fma(-c.y, pk.y, far[j]));
                }
                pk = cmul(pk, tau);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int yy = y0 + 4 * (2 * j + cls);
                pp.u[(size_t)(ly0 * 8 + yy) * n + lx0 * 8 + xx] += -far[j] * kInv2Pi;
            }
        }
        return;
    }
#pragma unroll 4
    for (int e = threadIdx.x; e < pw * pw; e += 256) {
        const int yy = e / pw, xx = e - yy * pw;
        const int lc = (yy >> 3) * tw + (xx >> 3);
        const double2 tau = make_double2(((xx & 7) - 3.5) * 0.125, ((yy & 7) - 3.5) * 0.125);
        double far = 0.0;
        double2 pk = make_double2(1.0, 0.0);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double2 c = sL[k * cnt + lc];
            far = fma(c.x, pk.x, fma(-c.y, pk.y, far));
            pk = cmul(pk, tau);
        }
        pp.u[(size_t)(ly0 * 8 + yy) * n + lx0 * 8 + xx] += -far * kInv2Pi;
    }
}

// one thread per point of the 8(K+1)-deep band (every point when the band
// covers the grid)
__global__ __launch_bounds__(256) void k_pass2_near(double *__restrict__ u,
                                                    const double *__restrict__ rq,
                                                    const double *__restrict__ rtab, int n, int nl,
                                                    int K, int kxp, int rs, RhsSet rh)
{
    if (!rhs_active(rh, blockIdx.z)) return;
    u += blockIdx.z * rh.sv;
    rq += blockIdx.z * rh.sr;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int B = 8 * (K + 1);
    int gx, gy;
    if (n <= 2 * B) {
        if (idx >= (int64_t)n * n) return;
        gx = (int)(idx % n);
        gy = (int)(idx / n);
    } else {
        const int64_t strip = (int64_t)B * n, side = (int64_t)B * (n - 2 * B);
        if (idx < strip) {
            gy = (int)(idx / n); gx = (int)(idx % n);
        } else if (idx < 2 * strip) {
            const int64_t i2 = idx - strip;
            gy = n - B + (int)(i2 / n); gx = (int)(i2 % n);
        } else if (idx < 2 * strip + side) {
            const int64_t i3 = idx - 2 * strip;
            gy = B + (int)(i3 / B); gx = (int)(i3 % B);
        } else if (idx < 2 * strip + 2 * side) {
            const int64_t i4 = idx - 2 * strip - side;
            gy = B + (int)(i4 / B); gx = n - B + (int)(i4 % B);
        } else {
            return;
        }
    }
    u[(size_t)gy * n + gx] += -pass2_near_at(gx, gy, rq, rtab, n, nl, K, kxp, rs) * kInv2Pi;
}

// ---------------------------------------------------------------------------
// host drivers.  Every launch covers the nr right-hand sides of rh in its
// third grid dimension.
// ---------------------------------------------------------------------------
template <int P>
static void run_m2m_from(fmm_plan *pl, double2 *M, int l_in, const RhsSet &rh, int nr, hipStream_t s)
{
    // each launch lifts the multipoles three levels, from l_in down to 2
    for (int l = l_in; l > 2; l -= 3) {
        const int nc = 1 << l, tw = std::min(nc, 8), nt = nc / tw;
        hipLaunchKernelGGL(k_m2m_up<P>, dim3(nt * nt, 1, nr), dim3(256), 0, s, M, pl->tab.m2m, pl->lv,
                           l, rh);
    }
}


// downward launches: (root level r, levels below it, root mode of k_down).
// Levels 2..L in chunks of three: trees with L <= 5 take one launch from the
// level-2 cells; deeper trees start at level 5, whose blocks build their own
// root from the ancestors (so levels 2..5 need no launch), then 8, 11, ...
struct DownChunk {
    int r, m, root;
};
static std::vector<DownChunk> down_chunks(int L)
{
    std::vector<DownChunk> ch;
    if (L <= 5) {
        ch.push_back({2, L - 2, 1});
        return ch;
    }
    for (int r = 5; r < L; r += 3) ch.push_back({r, std::min(3, L - r), r == 5 ? 2 : 0});
    return ch;
}

template <int P>
static int run_m2l_l2l(fmm_plan *pl, const double2 *M, double2 *Lm, double2 *Lt, const RhsSet &rh,
                       int nr, hipStream_t s, bool timed)
{
    const int rw = 16 + 4 * pl->K;
    const size_t shm = (size_t)P * rw * rw * sizeof(double2);
    const int ns = m2l_split_for(pl, nr);
    const int nitems = (int)pl->m2l_tiles.size() * ns;
    const M2LItem *items = pl->m2l_items[ns == 1 ? 0 : ns == 2 ? 1 : ns == 4 ? 2 : 3];
    if (nitems > 0) {
        StageTimer t(pl, timed ? FMM_STAGE_M2L : -1, s);
        // split 16-bit grid plans translate on the matrix cores, FP32 grid plans
        // in FP32; point clouds take only their near field in FP32 (Sec. 7.1)
        // and keep M2L in FP64
        const bool split16 = (pl->prec == FMM_SPLIT_FP16 || pl->prec == FMM_SPLIT_BF16) &&
                             pl->kind == FMM_GRID && pl->K == 1 && pl->nlist <= kM2L16MaxShare;
        if (split16) {
            const size_t shm16 = m2l16_lds<P>(rw);
            if (pl->prec == FMM_SPLIT_FP16)
                hipLaunchKernelGGL((k_m2l_mfma16<P, _Float16>), dim3(nitems, 1, nr), dim3(768), shm16, s,
                                   items, M, Lm, pl->lm_part, ns, pl->lv, pl->tab.m2lt16,
                                   pl->tab.m2l_off, pl->nlist, 2 * pl->K, rh);
            else
                hipLaunchKernelGGL((k_m2l_mfma16<P, __bf16>), dim3(nitems, 1, nr), dim3(768), shm16, s,
                                   items, M, Lm, pl->lm_part, ns, pl->lv, pl->tab.m2ltb16,
                                   pl->tab.m2l_off, pl->nlist, 2 * pl->K, rh);
        } else if (pl->prec != FMM_FP64 && pl->kind == FMM_GRID)
            hipLaunchKernelGGL((k_m2l<P, float>), dim3(nitems, 1, nr), dim3(kM2LThreads), shm / 2, s, items, M,
                               Lm, pl->lm_part, ns, pl->lv, pl->tab.hankl32, pl->tab.m2l_off, pl->tab.m2l_a,
                               pl->tab.m2l_b, pl->nlist, 2 * pl->K, rh);
        else
            hipLaunchKernelGGL((k_m2l<P, double>), dim3(nitems, 1, nr), dim3(kM2LThreads), shm, s, items, M,
                               Lm, pl->lm_part, ns, pl->lv, pl->tab.hankl, pl->tab.m2l_off, pl->tab.m2l_a,
                               pl->tab.m2l_b, pl->nlist, 2 * pl->K, rh);
    }
    StageTimer t(pl, timed ? FMM_STAGE_L2L : -1, s);
    for (const auto &c : down_chunks(pl->L))
        hipLaunchKernelGGL(k_down<P>, dim3(1 << (2 * c.r), 1, nr), dim3(256), 0, s, Lm, ns, pl->lm_part,
                           Lt,
                           pl->tab.l2l, pl->lv, c.r, c.m, c.root, rh);
    return FMM_OK;
}

static LeafArgs leaf_args(fmm_plan *pl, const double *q, double qscale, double *u,
                          const double2 *Lt, bool far, const RhsSet &rh)
{
    LeafArgs a;
    a.rh = rh;
    a.q = q;
    a.qscale = qscale;
    a.u = u;
    a.Lt = Lt;
    a.ktab = pl->tab.ktab;
    a.rtab = pl->tab.rtab;
    a.l2p = pl->tab.l2p;
    a.M = nullptr;
    a.p2m = pl->tab.p2m;
    a.lv = pl->lv;
    a.n = (int)pl->n;
    a.nl = pl->nl;
    a.L = pl->L;
    a.far = far ? 1 : 0;
    a.K = pl->K;
    a.kxp = near_kx_packed(pl);
    a.rs = 8 * pl->K + 9;
    return a;
}

// launches the leaf kernel of the plan's near radius (K >= 2: MAC theta)
template <int P>
static void launch_leaf_wide(fmm_plan *pl, dim3 gl, const LeafArgs &a, hipStream_t s)
{
    if constexpr (P <= kThetaPMax) {
        if (pl->K == 2) hipLaunchKernelGGL((k_leaf_wide<P, 2>), gl, dim3(512), 0, s, a);
        else if (pl->K == 3) hipLaunchKernelGGL((k_leaf_wide<P, 3>), gl, dim3(512), 0, s, a);
        else if (pl->K == 4) hipLaunchKernelGGL((k_leaf_wide<P, 4>), gl, dim3(512), 0, s, a);
    }
}

// FP32 plans with a MAC theta (K >= 2)
template <int P>
static void launch_leaf_wide_mfma32(fmm_plan *pl, dim3 gl, const LeafArgs &a, hipStream_t s)
{
    if constexpr (P <= kThetaPMax) {
        const float *kt = pl->tab.ktab32, *w = pl->tab.p2m32;
        if (pl->K == 2) hipLaunchKernelGGL((k_leaf_wide_mfma32<P, 2>), gl, dim3(256), 0, s, a, kt, w);
        else if (pl->K == 3) hipLaunchKernelGGL((k_leaf_wide_mfma32<P, 3>), gl, dim3(256), 0, s, a, kt, w);
        else if (pl->K == 4) hipLaunchKernelGGL((k_leaf_wide_mfma32<P, 4>), gl, dim3(256), 0, s, a, kt, w);
    }
}

template <int P>
static int grid_volume_fmm_p(fmm_plan *pl, const double *q, double qscale, double *u,
                             double *ring_out, bool defer_l2p, const RhsSet &rh, int nr,
                             hipStream_t s)
{
    const int nl = pl->nl;
    const bool far = pl->L >= 2;
    const bool fp32 = pl->prec == FMM_FP32;
    LeafArgs a = leaf_args(pl, q, qscale, u, pl->ws.Lt, far, rh);
    if (far) a.M = pl->ws.M;
    {
        StageTimer t(pl, FMM_STAGE_LEAF, s);
        dim3 gl((nl + 7) / 8, (nl + 7) / 8, nr);
        // split 16-bit plans: two blocks per compute unit over all right-hand
        // sides, each looping over tiles
        const int ntx = (nl + 7) / 8, ntiles = ntx * ntx;
        const dim3 g16(std::min(ntiles, std::max(1, (2 * pl->ncu + nr - 1) / nr)), 1, nr);
        if (pl->prec == FMM_SPLIT_FP16)
            hipLaunchKernelGGL((k_leaf_mfma16<P, _Float16>), g16, dim3(256), 0, s, a, pl->tab.ktab16,
                               pl->tab.p2m16, ntx, ntiles);
        else if (pl->prec == FMM_SPLIT_BF16)
            hipLaunchKernelGGL((k_leaf_mfma16<P, __bf16>), g16, dim3(256), 0, s, a, pl->tab.ktabb16,
                               pl->tab.p2mb16, ntx, ntiles);
        else if (fp32 && pl->K > 1)
            launch_leaf_wide_mfma32<P>(pl, gl, a, s);
        else if (fp32)
            hipLaunchKernelGGL(k_leaf_mfma32<P>, gl, dim3(256), 0, s, a, pl->tab.ktab32,
                               pl->tab.p2m32);
        else if (pl->K > 1)
            launch_leaf_wide<P>(pl, gl, a, s);
        else
            hipLaunchKernelGGL(k_leaf_grid<P>, gl, dim3(512), 0, s, a);
    }
    if (far) {
        {
            StageTimer t(pl, FMM_STAGE_M2M, s);
            run_m2m_from<P>(pl, pl->ws.M, pl->L, rh, nr, s);
        }
        run_m2l_l2l<P>(pl, pl->ws.M, pl->ws.Lm, pl->ws.Lt, rh, nr, s, true);
    }
    if (ring_out) {
        StageTimer t(pl, FMM_STAGE_RING, s);
        hipLaunchKernelGGL(k_ring_targets<P>, dim3(pl->n / 2, 1, nr), dim3(512), 0, s, a, ring_out,
                           pl->bem ? pl->bhat : nullptr);
    }
    if (far && !defer_l2p) {
        StageTimer t(pl, FMM_STAGE_L2L, s);
        const int tw = std::min(nl, 8);
        LeafArgs b = leaf_args(pl, nullptr, 1.0, u, nullptr, far, rh);
        hipLaunchKernelGGL(k_far_l2p<P>, dim3(nl / tw, nl / tw, nr), dim3(256), 0, s, b, nullptr,
                           nullptr, 0, pl->ws.Lt);
    }
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

template <int P>
static int grid_ring_source_fmm_p(fmm_plan *pl, double *u, bool with_volume, double *sigma_out,
                                  const RhsSet &rh, int nr, hipStream_t s)
{
    const int L = pl->L, nl = pl->nl;
    const bool far = L >= 2;
    StageTimer t(pl, FMM_STAGE_PASS2, s);
    if (far) {
        // upward: ring charges -> every boundary cell of levels 2..L
        const int tw = std::min(nl, 8);
        hipLaunchKernelGGL(k_p2m_ring<P>, dim3((pl->n_ring_p2m + 3) / 4, 1, nr), dim3(256), 0, s,
                           pl->ring_p2m_cells, pl->n_ring_p2m, pl->shat, pl->h, pl->ring_q,
                           sigma_out, pl->ws.M2, pl->lv, (int)pl->n, L, rh);
        // M2L from boundary cells into the (2K+2)-cell band of every level
        hipLaunchKernelGGL(k_m2l_ring<P>, dim3(pl->n_ring_cells, 1, nr), dim3(256), 0, s,
                           pl->ring_cells, pl->n_ring_cells, pl->ws.M2, pl->ws.Lm2, pl->lv,
                           pl->tab.hank, pl->tab.m2l_off, pl->tab.m2l_a, pl->tab.m2l_b,
                           pl->nlist, rh);
        // downward: levels 2..L-3 by k_down, the last three inside the far-field
        // kernel, whose blocks build their level-(L-3) root from the ancestors
        // when L - 3 <= 5 (then no k_down launch at all)
        const bool chain = L >= 5;
        const int last = chain ? L - 3 : L;
        const int chain_mode = !chain ? 0 : (last <= kMaxAncestorLevel ? 2 : 1);
        if (chain_mode != 2)
            for (const auto &c : down_chunks(last))
                hipLaunchKernelGGL(k_down<P>, dim3(1 << (2 * c.r), 1, nr), dim3(256), 0, s,
                                   pl->ws.Lm2, 1, (int64_t)0, pl->ws.Lt2, pl->tab.l2l, pl->lv, c.r, c.m, c.root,
                                   rh);
        const LeafArgs a = leaf_args(pl, nullptr, 1.0, u, pl->ws.Lt2, far, rh);
        hipLaunchKernelGGL(k_far_l2p<P>, dim3(nl / tw, nl / tw, nr), dim3(256), 0, s, a, pl->ws.Lm2,
                           pl->tab.l2l, chain_mode, with_volume ? pl->ws.Lt : nullptr);
    }
    const int n = (int)pl->n, B = 8 * (pl->K + 1);
    const int64_t nband = n <= 2 * B ? (int64_t)n * n : (int64_t)4 * B * n - 4 * B * B;
    hipLaunchKernelGGL(k_pass2_near, dim3((unsigned)((nband + 255) / 256), 1, nr), dim3(256), 0, s,
                       u, pl->ring_q, pl->tab.rtab, n, nl, pl->K, near_kx_packed(pl), 8 * pl->K + 9,
                       rh);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

int grid_volume_fmm(fmm_plan *pl, const double *q, double qscale, double *u, double *ring_out,
                    bool defer_l2p, const RhsSet &rh, int nr, hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, grid_volume_fmm_p, pl, q, qscale, u, ring_out, defer_l2p, rh, nr, s);
}

int grid_ring_source_fmm(fmm_plan *pl, double *u, bool with_volume, double *sigma_out,
                         const RhsSet &rh, int nr, hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, grid_ring_source_fmm_p, pl, u, with_volume, sigma_out, rh, nr, s);
}

template <int P>
static int tune_m2l_split_p(fmm_plan *pl, hipStream_t s, int *chosen)
{
    int st = ensure_rhs(pl, 1);
    if (st != FMM_OK) return st;
    if (pl->L < 2 || pl->m2l_tiles.empty()) {
        *chosen = pl->m2l_split;
        return FMM_OK;
    }
    // finite multipoles to translate (values do not affect the timing)
    FMM_HIP(pl, hipMemsetAsync(pl->ws.M, 0, (size_t)pl->exp_elems * sizeof(double2), s));
    const RhsSet rh = plan_rhs(pl, pl->kind == FMM_GRID ? (int64_t)pl->n * pl->n : (int64_t)pl->n,
                               nullptr);
    hipEvent_t e0, e1;
    FMM_HIP(pl, hipEventCreate(&e0));
    FMM_HIP(pl, hipEventCreate(&e1));
    // the fastest of three timed calls per split, over three rounds that
    // visit the splits in turn (so that a slow phase of the device does not
    // decide); ties go to the smaller split
    const int splits[4] = {1, 2, 4, 8};
    float split_ms[4] = {1e30f, 1e30f, 1e30f, 1e30f};
    for (int round = 0; round < 3 && st == FMM_OK; ++round)
        for (int i = 0; i < 4; ++i) {
            FMM_HIP(pl, hipStreamSynchronize(s));
            st = set_m2l_split(pl, splits[i]);
            if (st != FMM_OK) break;
            for (int rep = 0; rep < 4; ++rep) {
                FMM_HIP(pl, hipEventRecord(e0, s));
                run_m2l_l2l<P>(pl, pl->ws.M, pl->ws.Lm, pl->ws.Lt, rh, 1, s, false);
                FMM_HIP(pl, hipEventRecord(e1, s));
                FMM_HIP(pl, hipEventSynchronize(e1));
                float t = 0.0f;
                FMM_HIP(pl, hipEventElapsedTime(&t, e0, e1));
                if (rep > 0) split_ms[i] = std::min(split_ms[i], t);
            }
        }
    int best = pl->m2l_split;
    float best_ms = 1e30f;
    for (int i = 0; i < 4; ++i)
        if (split_ms[i] < best_ms) {
            best_ms = split_ms[i];
            best = splits[i];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FMM_OK) return st;
    st = set_m2l_split(pl, best);
    if (st == FMM_OK) *chosen = best;
    return st;
}

int tune_m2l_split(fmm_plan *pl, hipStream_t s, int *chosen)
{
    FMM_DISPATCH_P(pl->p, tune_m2l_split_p, pl, s, chosen);
}

// level-generic stages reused by point-cloud plans
template <int P>
static int points_up_p(fmm_plan *pl, hipStream_t s)
{
    StageTimer t(pl, FMM_STAGE_M2M, s);
    run_m2m_from<P>(pl, pl->ws.M, pl->L, RhsSet{}, 1, s);
    return FMM_OK;
}

template <int P>
static int points_down_p(fmm_plan *pl, hipStream_t s)
{
    return run_m2l_l2l<P>(pl, pl->ws.M, pl->ws.Lm, pl->ws.Lt, RhsSet{}, 1, s, true);
}

int points_upward_rest(fmm_plan *pl, hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, points_up_p, pl, s);
}

int points_m2l_down(fmm_plan *pl, hipStream_t s)
{
    FMM_DISPATCH_P(pl->p, points_down_p, pl, s);
}

// enable > 64 KB of dynamic LDS for the M2L kernels (gfx950 has 160 KB per CU)
template <int P>
static int m2l_attr_p(fmm_plan *pl)
{
    // the limit is a property of the kernel, shared by every plan of this p:
    // raise it to the largest tile any plan has needed so far
    static int high[kPMax + 1] = {0};
    const int rw = 16 + 4 * pl->K;
    const int shm = P * rw * rw * (int)sizeof(double2);
    if ((int64_t)shm > kM2LMaxLds) return fail(pl, FMM_ERR_UNSUPPORTED, "M2L source tile exceeds LDS");
    if (shm <= high[P]) return FMM_OK;
    FMM_HIP(pl, hipFuncSetAttribute((const void *)k_m2l<P, double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, shm));
    FMM_HIP(pl, hipFuncSetAttribute((const void *)k_m2l<P, float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, shm / 2));
    const int shm16 = (int)m2l16_lds<P>(rw);
    FMM_HIP(pl, hipFuncSetAttribute((const void *)k_m2l_mfma16<P, _Float16>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, shm16));
    FMM_HIP(pl, hipFuncSetAttribute((const void *)k_m2l_mfma16<P, __bf16>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, shm16));
    high[P] = shm;
    return FMM_OK;
}

int m2l_kernel_setup(fmm_plan *pl)
{
    FMM_DISPATCH_P(pl->p, m2l_attr_p, pl);
}

}  // namespace fmmprec
