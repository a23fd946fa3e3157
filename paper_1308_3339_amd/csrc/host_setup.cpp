// Host-side setup of a plan (plain C++, see host_setup.h).
//
// The operator tables follow the translation formulas of Sec. 5.3 of
// arXiv:1308.3339 rewritten for level-scaled expansions:
//   M2M (item 2):  M~par_n = -M~_0 c^n/n + sum_{k=1..n} 2^-k c^(n-k) C(n-1,k-1) M~_k,
//                  c = (child - parent centre)/w_parent
//   L2L (item 4):  L~child_n = 2^-n sum_{k>=n} C(k,n) c^(k-n) L~par_k
//   M2L (item 3):  Hankel generators H_0 = -log|d|, H_m = (m-1)!/d^m with
//                  d = target minus source centre in cell widths, and the
//                  scalings a_n = (-1)^n/n!, b_0 = -1, b_k = 1/(k-1)!
//   P2M (item 1) / L2P (item 5) on the fixed 8x8 leaf pattern,
//                  tau_j = (x_j - centre)/w_leaf
//   near field     T(d) = log(h |d|) on the integer lattice, T(0) = log(eps h)
#include "host_setup.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

namespace fmmprec {
namespace host {

using cd = std::complex<double>;

static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

static double binom(int a, int b)
{
    if (b < 0 || b > a) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return std::floor(r + 0.5);
}

static cd ipow(cd z, int k)
{
    cd r = 1.0;
    for (int i = 0; i < k; ++i) r *= z;
    return r;
}

bool in_near(double theta, int dx, int dy)
{
    if (theta <= 0.0) return dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1;
    return (double)(dx * dx + dy * dy) <= 2.0 / (theta * theta);
}

// Two cells of one level, radius r = w/sqrt2 each, are well separated when
// 2r < theta |d| w, i.e. |d|^2 > 2/theta^2; K is the largest k with (k, 0)
// not separated.  theta = 0 selects the list rule (K = 1).
int near_radius(double theta)
{
    if (theta <= 0.0) return 1;
    const double lim = 2.0 / (theta * theta);
    int k = 1;
    while ((double)((k + 1) * (k + 1)) <= lim) ++k;
    return k;
}

// split x = hi + lo with hi = fp16(x), lo = fp16(x - hi)
static void split16(double x, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)x;
    lo = (_Float16)(x - (double)hi);
}

// BF16 of x, rounded to nearest even on the FP32 bits
static __bf16 to_bf16(double x)
{
    const float f = (float)x;
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7fffu + ((b >> 16) & 1u);
    const uint16_t hb = (uint16_t)(b >> 16);
    __bf16 r;
    std::memcpy(&r, &hb, 2);
    return r;
}

static double bf16_val(__bf16 h)
{
    uint16_t hb;
    std::memcpy(&hb, &h, 2);
    const uint32_t b = (uint32_t)hb << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return (double)f;
}

static void splitb16(double x, __bf16 &hi, __bf16 &lo)
{
    hi = to_bf16(x);
    lo = to_bf16(x - bf16_val(hi));
}

bool build_tables(int p, double theta, double h, double self_eps, Tables &t, std::string &err)
{
    // M2M
    t.m2m.assign((size_t)4 * p * p, C2{0.0, 0.0});
    for (int qd = 0; qd < 4; ++qd) {
        const cd c(0.5 * ((qd & 1) - 0.5), 0.5 * ((qd >> 1) - 0.5));
        for (int n = 0; n < p; ++n)
            for (int k = 0; k <= n; ++k) {
                cd v;
                if (n == 0) v = 1.0;
                else if (k == 0) v = -ipow(c, n) / (double)n;
                else v = std::ldexp(1.0, -k) * ipow(c, n - k) * binom(n - 1, k - 1);
                t.m2m[((size_t)qd * p + n) * p + k] = C2{v.real(), v.imag()};
            }
    }
    // L2L: L~child_n = sum_{k>=n} C(k,n) c^(k-n) 2^-n L~parent_k
    t.l2l.assign((size_t)4 * p * p, C2{0.0, 0.0});
    for (int qd = 0; qd < 4; ++qd) {
        const cd c(0.5 * ((qd & 1) - 0.5), 0.5 * ((qd >> 1) - 0.5));
        for (int n = 0; n < p; ++n)
            for (int k = n; k < p; ++k) {
                const cd v = binom(k, n) * ipow(c, k - n) * std::ldexp(1.0, -n);
                t.l2l[((size_t)qd * p + n) * p + k] = C2{v.real(), v.imag()};
            }
    }
    // M2L Hankel generators for source offsets (dx, dy) in [-R, R]^2, R =
    // 2K + 1 (source cell = target cell + (dx, dy)); the expansion variable
    // of Sec. 5.3 is z_{Lambda M} = target centre - source centre = -(dx + i dy)
    // cell widths.  Offsets of the near disk are never used.
    const int nh = 2 * p - 1, K = near_radius(theta), R = 2 * K + 1, RD = 2 * R + 1;
    t.hank.assign((size_t)RD * RD * nh, C2{0.0, 0.0});
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            if (in_near(theta, dx, dy)) continue;
            const cd d(-(double)dx, -(double)dy);
            const size_t o = (size_t)((dy + R) * RD + dx + R) * nh;
            t.hank[o] = C2{-std::log(std::abs(d)), 0.0};
            for (int m = 1; m < nh; ++m) {
                const cd v = factorial(m - 1) / ipow(d, m);
                t.hank[o + m] = C2{v.real(), v.imag()};
            }
        }
    // interaction-list offsets per parity class: children of the parent's
    // near set that are not in the target's own near set (Sec. 5.2; with the
    // 3x3 near set of the list rule these are the 27 of the paper's Fig. 3,
    // with a MAC theta the traversal's equivalent lists on the uniform tree)
    std::vector<std::vector<I4>> cls(4);
    for (int w = 0; w < 4; ++w) {
        const int px = w & 1, py = w >> 1;
        for (int dy = -2 * K - py; dy <= 2 * K + 1 - py; ++dy)
            for (int dx = -2 * K - px; dx <= 2 * K + 1 - px; ++dx) {
                if (in_near(theta, dx, dy)) continue;
                // parent offset of the source
                const int Dx = (dx + px) >> 1, Dy = (dy + py) >> 1;
                if (!in_near(theta, Dx, Dy)) continue;
                cls[w].push_back(I4{dx, dy, (dy + R) * RD + dx + R, 0});
            }
    }
    for (int w = 1; w < 4; ++w)
        if (cls[w].size() != cls[0].size()) {
            err = "internal: interaction list size";
            return false;
        }
    t.nlist = (int)cls[0].size();
    if (K == 1 && t.nlist != 27) {
        err = "internal: interaction list size";
        return false;
    }
    t.offs.clear();
    for (int w = 0; w < 4; ++w) t.offs.insert(t.offs.end(), cls[w].begin(), cls[w].end());
    // the generators again in list order, [class][list entry][2p - 1], so
    // that M2L finds an entry's generators without first loading its offset
    t.hankl.assign(t.offs.size() * (size_t)nh, C2{0.0, 0.0});
    for (size_t e = 0; e < t.offs.size(); ++e)
        for (int m = 0; m < nh; ++m) t.hankl[e * nh + m] = t.hank[(size_t)t.offs[e].z * nh + m];
    t.an.assign(p, 0.0);
    t.bk.assign(p, 0.0);
    for (int k = 0; k < p; ++k) {
        t.an[k] = ((k & 1) ? -1.0 : 1.0) / factorial(k);
        t.bk[k] = (k == 0) ? -1.0 : 1.0 / factorial(k - 1);
    }
    // leaf point pattern
    t.p2m.assign((size_t)p * 64, C2{0.0, 0.0});
    t.l2p.assign((size_t)64 * p, C2{0.0, 0.0});
    for (int j = 0; j < 64; ++j) {
        const int a = j & 7, b = j >> 3;
        const cd tau((a - 3.5) / 8.0, (b - 3.5) / 8.0);
        for (int k = 0; k < p; ++k) {
            const cd pk = ipow(tau, k);
            const cd w = (k == 0) ? cd(1.0) : -pk / (double)k;
            t.p2m[(size_t)k * 64 + j] = C2{w.real(), w.imag()};
            t.l2p[(size_t)j * p + k] = C2{pk.real(), pk.imag()};
        }
    }
    // near-field kernel table: lattice offsets within the (2K+1)^2 leaves
    // around a leaf, |dx|, |dy| <= 8K + 7 (side 31 for K = 1)
    const int KC = 8 * K + 7, KS = 2 * KC + 1;
    t.kt.assign((size_t)KS * KS, 0.0);
    for (int dy = -KC; dy <= KC; ++dy)
        for (int dx = -KC; dx <= KC; ++dx) {
            const double v = (dx == 0 && dy == 0)
                                 ? std::log(self_eps * h)
                                 : std::log(h * std::sqrt((double)(dx * dx + dy * dy)));
            t.kt[(size_t)(dy + KC) * KS + dx + KC] = v;
        }
    // ring node to grid node: |dx|, |dy| <= 8(K + 1) (side 17 for K = 1)
    const int RS = 8 * K + 9;
    t.rt.assign((size_t)RS * RS, 0.0);
    for (int dy = 0; dy < RS; ++dy)
        for (int dx = 0; dx < RS; ++dx)
            if (dx || dy) t.rt[(size_t)dy * RS + dx] = std::log(h * std::sqrt((double)(dx * dx + dy * dy)));
    // FP32 and split-FP16 tables (the split-FP16 leaf kernel exists for the 3x3 near set only)
    t.kt32.assign(t.kt.begin(), t.kt.end());
    const int prow = 16 * ((2 * p + 15) / 16);
    t.p2m32.assign((size_t)prow * 64, 0.0f);
    t.p2m16.assign((size_t)2 * prow * 64, (_Float16)0.0f);
    for (int k = 0; k < p; ++k)
        for (int j = 0; j < 64; ++j) {
            t.p2m32[(size_t)(2 * k) * 64 + j] = (float)t.p2m[(size_t)k * 64 + j].x;
            t.p2m32[(size_t)(2 * k + 1) * 64 + j] = (float)t.p2m[(size_t)k * 64 + j].y;
        }
    t.p2mb16.assign((size_t)2 * prow * 64, to_bf16(0.0));
    for (int r = 0; r < 2 * p; ++r)
        for (int j = 0; j < 64; ++j) {
            const C2 w = t.p2m[(size_t)(r / 2) * 64 + j];
            split16(r & 1 ? w.y : w.x, t.p2m16[(size_t)r * 64 + j], t.p2m16[(size_t)(prow + r) * 64 + j]);
            splitb16(r & 1 ? w.y : w.x, t.p2mb16[(size_t)r * 64 + j],
                     t.p2mb16[(size_t)(prow + r) * 64 + j]);
        }
    // kernel table in 8 column-shifted copies: copy c, row r, entry j = T[r][j + c]
    // (the 3x3 near set's 31 x 31 table; a wider table's first 31 columns
    // and rows otherwise, which no split-FP16 plan reads)
    t.kt16.assign((size_t)2 * 8 * 31 * 40, (_Float16)0.0f);
    t.ktb16.assign((size_t)2 * 8 * 31 * 40, to_bf16(0.0));
    for (int c = 0; c < 8; ++c)
        for (int r = 0; r < 31; ++r)
            for (int j = 0; j + c <= 30 && j < 40; ++j) {
                const double v = t.kt[(size_t)r * KS + j + c];
                split16(v, t.kt16[((size_t)c * 31 + r) * 40 + j], t.kt16[((size_t)(8 + c) * 31 + r) * 40 + j]);
                splitb16(v, t.ktb16[((size_t)c * 31 + r) * 40 + j], t.ktb16[((size_t)(8 + c) * 31 + r) * 40 + j]);
            }
    // matrix-core M2L operators (see Tables::m2lt16)
    t.m2l_mp = 16 * ((2 * p + 15) / 16);
    t.m2l_kp = 8 * ((2 * p + 7) / 8);
    const size_t nent = t.offs.size(), esz = (size_t)t.m2l_mp * t.m2l_kp;
    t.m2lt16.assign(2 * nent * esz, (_Float16)0.0f);
    t.m2ltb16.assign(2 * nent * esz, to_bf16(0.0));
    for (size_t e = 0; e < nent; ++e)
        for (int nn = 0; nn < p; ++nn)
            for (int k = 0; k < p; ++k) {
                const C2 hv = t.hankl[e * nh + nn + k];
                const cd tv = t.an[nn] * cd(hv.x, hv.y) * t.bk[k];
                // (Re L, Im L) += [[Re T, -Im T], [Im T, Re T]] (Re M, Im M)
                const double v[2][2] = {{tv.real(), -tv.imag()}, {tv.imag(), tv.real()}};
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 2; ++c) {
                        const size_t i = e * esz + (size_t)(2 * nn + r) * t.m2l_kp + 2 * k + c;
                        split16(v[r][c], t.m2lt16[i], t.m2lt16[nent * esz + i]);
                        splitb16(v[r][c], t.m2ltb16[i], t.m2ltb16[nent * esz + i]);
                    }
            }
    t.hank32.resize(t.hank.size());
    t.hankl32.resize(t.hankl.size());
    for (size_t i = 0; i < t.hank.size(); ++i) t.hank32[i] = F2{(float)t.hank[i].x, (float)t.hank[i].y};
    for (size_t i = 0; i < t.hankl.size(); ++i) t.hankl32[i] = F2{(float)t.hankl[i].x, (float)t.hankl[i].y};
    return true;
}

void build_work(int L, int p, int K, double side, bool ring_lists, Work &w)
{
    int64_t off = 0;
    for (int l = 0; l <= kMaxLevelsH; ++l) {
        w.off[l] = 0;
        w.logw[l] = 0.0;
    }
    for (int l = 2; l <= L; ++l) {
        w.off[l] = off;
        off += ((int64_t)1 << (2 * l)) * p;
        w.logw[l] = std::log(side / (double)(1 << l));
    }
    w.exp_elems = off;
    w.tiles.clear();
    w.ring.clear();
    w.ring_p2m.clear();
    for (int l = L; l >= 2; --l) {
        const int nc = 1 << l, tw = std::min(16, nc), nt = nc / tw;
        for (int ty = 0; ty < nt; ++ty)
            for (int tx = 0; tx < nt; ++tx) w.tiles.push_back(I4{l, 0, tx * tw, ty * tw});
        if (!ring_lists) continue;
        // strips of cells whose lists can hold a boundary cell of level l (those
        // within 2K + 1 cells of the boundary): (level, side | depth << 2,
        // start, end), 64 lanes per item stepping by 2 from start
        const int band = 2 * K + 2;
        if (nc <= 2 * band) {
            for (int d = 0; d < nc; ++d)
                for (int par = 0; par < 2; ++par) w.ring.push_back(I4{l, 0 | (d << 2), par, nc});
        } else {
            for (int s = 0; s < 4; ++s)
                for (int d = 0; d < band; ++d)
                    for (int par = 0; par < 2; ++par) {
                        const int lo = (s & 1) ? band : 0, hi = (s & 1) ? nc - band : nc;
                        for (int a0 = lo + par; a0 < hi; a0 += 128) w.ring.push_back(I4{l, s | (d << 2), a0, hi});
                    }
        }
    }
    if (!ring_lists) return;
    // boundary cells of every level: targets of the ring charges' P2M
    for (int l = 2; l <= L; ++l) {
        const int nc = 1 << l;
        for (int iy = 0; iy < nc; ++iy)
            for (int ix = 0; ix < nc; ++ix)
                if (ix == 0 || iy == 0 || ix == nc - 1 || iy == nc - 1) w.ring_p2m.push_back(I4{l, ix, iy, 0});
    }
}

// tile by tile, the shares of one tile next to each other (they read the
// same sources, which then come from L2)
std::vector<I4> m2l_items(const std::vector<I4> &tiles, int split)
{
    std::vector<I4> items;
    items.reserve(tiles.size() * split);
    for (const I4 &t : tiles)
        for (int part = 0; part < split; ++part) items.push_back(I4{t.x, part, t.z, t.w});
    return items;
}

int default_m2l_split(int tiles, int ncu)
{
    int split = 1;
    while (split < 8 && (int64_t)2 * split * tiles < ncu) split *= 2;
    return split;
}

}  // namespace host
}  // namespace fmmprec
