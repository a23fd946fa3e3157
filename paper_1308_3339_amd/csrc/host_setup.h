// Host-side setup of a plan: the operator tables, the interaction lists, the
// level layout and the work lists of the kernels.  Plain C++ (no HIP): the
// library uploads what these functions build, and the host sanitizer check
// (tests/sanitize/host_setup_check.cpp) builds and checks the same tables
// under AddressSanitizer and UndefinedBehaviorSanitizer.
#ifndef FMMPREC_HOST_SETUP_H
#define FMMPREC_HOST_SETUP_H

#include <cstdint>
#include <string>
#include <vector>

namespace fmmprec {
namespace host {

// layouts of the device vector types the tables are uploaded into
struct C2 {
    double x, y;
};
struct F2 {
    float x, y;
};
struct I4 {
    int32_t x, y, z, w;
};

constexpr int kMaxLevelsH = 24;
constexpr int kMaxKH = 4;

// Near set of a leaf (Sec. 5.2): the 3x3 leaves of the list rule (theta <= 0),
// or with a MAC theta the disk |d|^2 <= 2 / theta^2 of the dual tree
// traversal on the uniform tree.
bool in_near(double theta, int dx, int dy);
// its radius K in leaves (1 for the list rule)
int near_radius(double theta);

// Operator tables of one p and near set (Sec. 5.3, level-scaled): see
// build_tables for the layouts.
struct Tables {
    std::vector<C2> m2m, l2l;     // [4 quadrants][p][p]
    std::vector<C2> hank;         // [(2R+1)^2 offsets][2p-1], R = 2K+1
    std::vector<C2> hankl;        // [4 classes][nlist][2p-1], list order
    std::vector<I4> offs;         // [4 classes][nlist]: (dx, dy, hank index, 0)
    int nlist = 0;
    std::vector<double> an, bk;   // M2L output / input scalings
    std::vector<C2> p2m, l2p;     // [p][64] and [64][p] on the 8x8 leaf pattern
    std::vector<double> kt;       // near-field log table, side 16K+15
    std::vector<double> rt;       // ring node to grid node, side 8K+9
    std::vector<float> kt32, p2m32;
    std::vector<_Float16> kt16, p2m16;   // split FP16 halves
    std::vector<__bf16> ktb16, p2mb16;   // split BF16 halves
    std::vector<F2> hank32, hankl32;
    // M2L operators of the list entries for the split 16-bit matrix-core
    // M2L: entry e of class w as the real 2p x 2p matrix of
    //   L~_n = sum_k a_n H_{n+k} b_k M~_k      (H_0 without the level's log w)
    // rows 2n + {Re, Im}, columns 2k + {Re, Im} of M~_k, padded to m2l_mp
    // rows and m2l_kp columns; [w][e][m2l_mp][m2l_kp] halves, the hi parts,
    // then the lo parts (x = hi + lo)
    int m2l_mp = 0, m2l_kp = 0;
    std::vector<_Float16> m2lt16;
    std::vector<__bf16> m2ltb16;
};

// Fills t; returns false with a message in err when the interaction lists
// come out inconsistent (an internal error).
bool build_tables(int p, double theta, double h, double self_eps, Tables &t, std::string &err);

// Level layout and work lists of a tree with L levels below the root.
struct Work {
    int64_t off[kMaxLevelsH + 1];   // double2 offset of level l in an expansion buffer
    double logw[kMaxLevelsH + 1];   // log(cell width) at level l
    int64_t exp_elems = 0;          // double2 elements per expansion buffer
    std::vector<I4> tiles;          // M2L tiles: (level, 0, tx0, ty0), 16x16 cells or the level
    std::vector<I4> ring;           // strips next to the boundary (k_m2l_ring)
    std::vector<I4> ring_p2m;       // boundary cells of levels 2..L: (level, ix, iy, 0)
};

void build_work(int L, int p, int K, double side, bool ring_lists, Work &w);

// the M2L work items of split S: every tile S times, part 0..S-1
std::vector<I4> m2l_items(const std::vector<I4> &tiles, int split);

// the smallest split in {1, 2, 4, 8} that gives half the compute units a block
int default_m2l_split(int tiles, int ncu);

}  // namespace host
}  // namespace fmmprec

#endif
