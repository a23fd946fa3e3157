// Host sanitizer check of the library's setup code (csrc/host_setup.cpp),
// built with -fsanitize=address,undefined by tests/test_sanitizers.py and
// run on the CPU.  It builds the operator tables, interaction lists and
// work lists for every supported p, several near sets and tree depths, and
// checks properties of each against what Secs. 5.2-5.3 fix:
//   * the list rule gives 27 interaction-list entries per parity class, a
//     MAC theta the same count in every class, every entry outside the near
//     set with its parent inside the parent's near set;
//   * the generators of an entry are those of its offset, all finite;
//   * the near-field log table is symmetric under the lattice symmetries;
//   * M2M is lower triangular and P2M's first row is the charge sum;
//   * the M2L tiles cover every cell of levels 2..L once; the items of a
//     split carry every share of every tile; the boundary strips and
//     boundary cells stay inside their levels.
// Any out-of-bounds access or undefined behaviour stops it through the
// sanitizers; a failed property makes it exit with status 1.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "host_setup.h"

using namespace fmmprec::host;

static int failures = 0;

#define CHECK(cond, ...)                              \
    do {                                              \
        if (!(cond)) {                                \
            std::printf("FAIL %s: ", #cond);          \
            std::printf(__VA_ARGS__);                 \
            std::printf("\n");                        \
            ++failures;                               \
        }                                             \
    } while (0)

static bool finite(const C2 &c) { return std::isfinite(c.x) && std::isfinite(c.y); }

static void check_tables(int p, double theta, int n)
{
    const double h = 1.0 / (n + 1);
    Tables t;
    std::string err;
    const bool ok = build_tables(p, theta, h, 0.1985, t, err);
    CHECK(ok, "p=%d theta=%g: %s", p, theta, err.c_str());
    if (!ok) return;
    const int K = near_radius(theta), R = 2 * K + 1, RD = 2 * R + 1, nh = 2 * p - 1;
    if (theta <= 0.0) CHECK(t.nlist == 27, "list rule nlist %d", t.nlist);
    CHECK((int)t.offs.size() == 4 * t.nlist, "offs size");
    for (int w = 0; w < 4; ++w) {
        const int px = w & 1, py = w >> 1;
        for (int e = 0; e < t.nlist; ++e) {
            const I4 o = t.offs[(size_t)w * t.nlist + e];
            CHECK(!in_near(theta, o.x, o.y), "entry in the near set p=%d theta=%g", p, theta);
            CHECK(in_near(theta, (o.x + px) >> 1, (o.y + py) >> 1), "parent not near");
            CHECK(o.z == (o.y + R) * RD + o.x + R, "hank index");
            for (int m = 0; m < nh; ++m) {
                const C2 a = t.hankl[((size_t)w * t.nlist + e) * nh + m];
                const C2 b = t.hank[(size_t)o.z * nh + m];
                CHECK(a.x == b.x && a.y == b.y, "list-order generators differ");
                CHECK(finite(a), "generator not finite");
            }
        }
    }
    const int KC = 8 * K + 7, KS = 2 * KC + 1;
    CHECK((int)t.kt.size() == KS * KS, "kt size");
    for (int dy = -KC; dy <= KC; ++dy)
        for (int dx = -KC; dx <= KC; ++dx) {
            const double v = t.kt[(size_t)(dy + KC) * KS + dx + KC];
            CHECK(std::isfinite(v), "kt not finite");
            CHECK(v == t.kt[(size_t)(-dy + KC) * KS - dx + KC], "kt not symmetric under d -> -d");
            CHECK(v == t.kt[(size_t)(dx + KC) * KS + dy + KC], "kt not symmetric under transpose");
        }
    for (int qd = 0; qd < 4; ++qd)
        for (int nn = 0; nn < p; ++nn)
            for (int k = nn + 1; k < p; ++k) {
                const C2 c = t.m2m[((size_t)qd * p + nn) * p + k];
                CHECK(c.x == 0.0 && c.y == 0.0, "M2M not lower triangular");
            }
    for (int j = 0; j < 64; ++j) CHECK(t.p2m[j].x == 1.0 && t.p2m[j].y == 0.0, "P2M row 0");
    CHECK(t.an[0] == 1.0 && t.bk[0] == -1.0, "M2L scalings");
    for (const C2 &c : t.l2p) CHECK(finite(c), "L2P not finite");
    for (float v : t.kt32) CHECK(std::isfinite(v), "FP32 table not finite");
}

static void check_work(int L, int p, int K)
{
    Work w;
    build_work(L, p, K, 1.0, true, w);
    int64_t elems = 0;
    for (int l = 2; l <= L; ++l) {
        CHECK(w.off[l] == elems, "level offset L=%d l=%d", L, l);
        elems += ((int64_t)1 << (2 * l)) * p;
    }
    CHECK(w.exp_elems == elems, "expansion size");
    for (int l = 2; l <= L; ++l) {
        const int nc = 1 << l;
        std::vector<int> cover((size_t)nc * nc, 0);
        for (const I4 &t : w.tiles) {
            if (t.x != l) continue;
            const int tw = nc < 16 ? nc : 16;
            for (int y = 0; y < tw; ++y)
                for (int x = 0; x < tw; ++x) {
                    const int cx = t.z + x, cy = t.w + y;
                    CHECK(cx >= 0 && cx < nc && cy >= 0 && cy < nc, "tile outside level");
                    if (cx >= 0 && cx < nc && cy >= 0 && cy < nc) ++cover[(size_t)cy * nc + cx];
                }
        }
        for (int c : cover) CHECK(c == 1, "cell covered %d times at level %d", c, l);
    }
    for (const I4 &r : w.ring) {
        const int l = r.x, nc = 1 << l;
        CHECK(l >= 2 && l <= L, "strip level");
        CHECK(r.z >= 0 && r.z < r.w && r.w <= nc, "strip range");
        CHECK((r.y >> 2) < nc, "strip depth");
    }
    int64_t nb = 0;
    for (int l = 2; l <= L; ++l) nb += 4 * (1 << l) - 4;
    CHECK((int64_t)w.ring_p2m.size() == (L >= 2 ? nb : 0), "boundary cells");
    for (int split : {1, 2, 4, 8}) {
        const std::vector<I4> items = m2l_items(w.tiles, split);
        CHECK(items.size() == w.tiles.size() * split, "items");
        for (size_t i = 0; i < items.size(); ++i) {
            const I4 &t = w.tiles[i / split];
            CHECK(items[i].y == (int)(i % split) && items[i].x == t.x && items[i].z == t.z &&
                      items[i].w == t.w,
                  "item %zu", i);
        }
    }
    const int s = default_m2l_split((int)w.tiles.size(), 256);
    CHECK(s == 1 || s == 2 || s == 4 || s == 8, "default split");
}

int main()
{
    const double thetas[] = {0.0, 0.3, 0.4, 0.5, 0.6, 0.8};
    int configs = 0;
    for (int p = 2; p <= 20; ++p)
        for (double th : thetas)
            for (int n : {8, 64, 2048}) {
                check_tables(p, th, n);
                ++configs;
            }
    for (int L = 0; L <= 9; ++L)
        for (int K = 1; K <= kMaxKH; ++K)
            for (int p : {2, 10}) {
                check_work(L, p, K);
                ++configs;
            }
    std::printf("%d configurations, %d failures\n", configs, failures);
    if (failures == 0) std::printf("host setup check ok\n");
    return failures == 0 ? 0 : 1;
}
