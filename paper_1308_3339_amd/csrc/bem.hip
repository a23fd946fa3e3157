// Boundary correction of the FMM-BEM preconditioner (Sec. 4.1 and 4.3 of
// arXiv:1308.3339) for zero Dirichlet data.
//
// Collocation at the 4n ring nodes with constant elements of length h:
//   S_kl = h G(|y_k - y_l|) (k != l),  S_kk = -(h/2pi)(log(h/2) - 1),
// and the density solves S sigma = -phi_ring.
//
// The ring is invariant under the 90-degree rotation of the square, which
// maps node (side s, k) to (s+1, k).  S is therefore block circulant,
// S_{s,s'} = C_{(s'-s) mod 4}, and the 4-point DFT over sides diagonalises
// it into S^_m = sum_r C_r i^(mr):
//   S^_0 = C0 + C1 + C2 + C3 (real),  S^_2 = C0 - C1 + C2 - C3 (real),
//   S^_1 = (C0 - C2) + i (C1 - C3) (Hermitian),  S^_3 = conj(S^_1).
// All three are Hermitian positive definite (S is SPD), so they are inverted
// once at setup by Gauss-Jordan without pivoting.
//
// The ring is also invariant under the reflections of the square, which
// reverse the node order along a side (J: k -> n-1-k) and map side s to -s.
// Hence J S^_0 J = S^_0, J S^_2 J = S^_2 and J S^_1 J = conj(S^_1), and the
// same holds for the inverses X_m.  In the even/odd basis of each side,
// Q = [[I, J], [I, -J]] on the two halves of the side, the real blocks split
// into two (n/2)^2 blocks and the complex one into four real (n/2)^2 blocks
// (its real part maps even to even and odd to odd, its imaginary part even to
// odd and odd to even).  Setup folds the inverses into these eight halves
// (each averaged over the four symmetric copies of its entries, with the 1/2
// of Q^T Q = 2 I), and an application is a DFT over the sides with the
// even/odd split (formed by the ring-target kernel of the volume pass), eight
// (n/2) x (n/2) products (here) and the inverse (formed where the
// boundary-source pass reads the density): 2n^2 doubles read, against 4n^2
// for the rotation blocks alone and 16n^2 for a dense inverse.
#include "fmm_internal.h"

namespace fmmprec {

__device__ __forceinline__ void ring_xy(int t, int n, int &Ix, int &Iy)
{
    const int s = t / n, k = t - s * n;
    if (s == 0) { Ix = k + 1; Iy = 0; }
    else if (s == 1) { Ix = n + 1; Iy = k + 1; }
    else if (s == 2) { Ix = n - k; Iy = n + 1; }
    else { Ix = 0; Iy = n - k; }
}

// S^_0, S^_2 (real) and S^_1 (complex) for rows k (bottom side) and columns k'
__global__ __launch_bounds__(256) void k_bem_build(double *__restrict__ S0,
                                                   double *__restrict__ S2,
                                                   double2 *__restrict__ S1, int n)
{
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const double h = 1.0 / (double)(n + 1);
    int xi, yi;
    ring_xy(i, n, xi, yi);
    double C[4];
    for (int r = 0; r < 4; ++r) {
        int xj, yj;
        ring_xy(r * n + j, n, xj, yj);
        if (r == 0 && i == j) {
            C[r] = -(h * kInv2Pi) * (log(0.5 * h) - 1.0);
        } else {
            const double dx = (double)(xi - xj), dy = (double)(yi - yj);
            C[r] = -(h * kInv2Pi) * log(h * sqrt(dx * dx + dy * dy));
        }
    }
    const size_t e = (size_t)i * n + j;
    S0[e] = (C[0] + C[1]) + (C[2] + C[3]);
    S2[e] = (C[0] - C[1]) + (C[2] - C[3]);
    S1[e] = make_double2(C[0] - C[2], C[1] - C[3]);
}

// Blocked Gauss-Jordan inversion in place, without pivoting (the blocks are
// Hermitian positive definite), in panels of kGjB columns.  With K the
// panel's index range, D = A[K,K], C = A[:,K] and R = D^-1 A[K,:]:
//   A[K,K] <- D^-1,  A[K,j] <- R[:,j],  A[i,K] <- -C[i,:] D^-1,
//   A[i,j] <- A[i,j] - C[i,:] R[:,j]          (i, j outside K),
// i.e. kGjB unblocked elimination steps at once.  R[:,K] holds D^-1, so the
// rows i outside K take A[i,j] <- [j outside K] A[i,j] - C[i,:] R[:,j] for
// every column.  Three launches per panel: D^-1 by one block in LDS, then R
// and a copy of C, then the rank-kGjB update (64 x 64 output tiles).
constexpr int kGjB = 32;

// complex entries as a clang vector of (re, im), the layout of double2
typedef double gj_c __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double gj_mul(double a, double b) { return a * b; }
__device__ __forceinline__ gj_c gj_mul(gj_c a, gj_c b)
{
    return gj_c{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double gj_fms(double acc, double a, double b) { return fma(-a, b, acc); }
__device__ __forceinline__ gj_c gj_fms(gj_c acc, gj_c a, gj_c b)
{
    return gj_c{fma(-a.x, b.x, fma(a.y, b.y, acc.x)), fma(-a.x, b.y, fma(-a.y, b.x, acc.y))};
}
__device__ __forceinline__ double gj_inv(double a) { return 1.0 / a; }
__device__ __forceinline__ gj_c gj_inv(gj_c a)
{
    const double d = a.x * a.x + a.y * a.y;
    return gj_c{a.x / d, -a.y / d};
}
template <typename T> __device__ __forceinline__ T gj_zero();
template <> __device__ __forceinline__ double gj_zero<double>() { return 0.0; }
template <> __device__ __forceinline__ gj_c gj_zero<gj_c>() { return gj_c{0.0, 0.0}; }
__device__ __forceinline__ double gj_neg(double a) { return -a; }
__device__ __forceinline__ gj_c gj_neg(gj_c a) { return -a; }

// D^-1 of the diagonal block at k0 (b = min(kGjB, n) rows) into Dinv [b][b],
// by b unpivoted elimination steps in LDS
template <typename T>
__global__ __launch_bounds__(256) void k_gj_diag(const T *__restrict__ A, T *__restrict__ Dinv, int n,
                                                 int k0, int b)
{
    __shared__ T D[kGjB][kGjB + 1];
    for (int e = threadIdx.x; e < b * b; e += 256) D[e / b][e % b] = A[(size_t)(k0 + e / b) * n + k0 + e % b];
    __syncthreads();
    constexpr int NQ = kGjB * kGjB / 256;   // elements per thread at b = kGjB
    for (int k = 0; k < b; ++k) {
        const T ip = gj_inv(D[k][k]);
        T v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = threadIdx.x + 256 * q;
            if (e >= b * b) continue;
            const int r = e / b, c = e % b;
            if (r == k) v[q] = c == k ? ip : gj_mul(D[k][c], ip);
            else if (c == k) v[q] = gj_neg(gj_mul(D[r][k], ip));
            else v[q] = gj_fms(D[r][c], gj_mul(D[r][k], ip), D[k][c]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = threadIdx.x + 256 * q;
            if (e < b * b) D[e / b][e % b] = v[q];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < b * b; e += 256) Dinv[e] = D[e / b][e % b];
}

// R [b][n] = D^-1 A[K,:] (D^-1 itself in the panel's columns), a thread
// per (r, j): r = 4 blockIdx.y + wave, j = 64 blockIdx.x + lane; the blocks
// of blockIdx.y = 0 also copy the column panel C [n][b] = A[:,K]
template <typename T>
__global__ __launch_bounds__(256) void k_gj_panel(const T *__restrict__ A, const T *__restrict__ Dinv,
                                                  T *__restrict__ R, T *__restrict__ C, int n, int k0,
                                                  int b)
{
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    if (r < b) {
        T v;
        if (j >= k0 && j < k0 + b) {
            v = Dinv[r * b + j - k0];
        } else {
            v = gj_zero<T>();
            for (int s = 0; s < b; ++s) v = gj_fms(v, gj_neg(Dinv[r * b + s]), A[(size_t)(k0 + s) * n + j]);
        }
        R[(size_t)r * n + j] = v;
    }
    if (blockIdx.y == 0 && (threadIdx.x >> 6) == 0)
        for (int s = 0; s < b; ++s) C[(size_t)j * b + s] = A[(size_t)j * n + k0 + s];
}

// rows per thread of the update tile: 4 (real), 2 (complex)
template <typename T> constexpr int gj_rows() { return sizeof(T) == sizeof(double) ? 4 : 2; }

// A <- the panel's elimination, (16 TI) x 64 output tiles (a thread TI x 4
// of them), C and R tiles in LDS
template <typename T>
__global__ __launch_bounds__(256) void k_gj_update(T *__restrict__ A, const T *__restrict__ R,
                                                   const T *__restrict__ C, int n, int k0, int b)
{
    constexpr int TI = gj_rows<T>(), TR = 16 * TI;
    __shared__ T sc[TR][kGjB + 1], sr[kGjB][64];
    const int i0 = blockIdx.y * TR, j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int e = threadIdx.x; e < TR * b; e += 256) {
        const int r = e / b, s = e % b;
        sc[r][s] = i0 + r < n ? C[(size_t)(i0 + r) * b + s] : gj_zero<T>();
    }
    for (int e = threadIdx.x; e < 64 * b; e += 256) {
        const int s2 = e / 64, c = e % 64;
        sr[s2][c] = j0 + c < n ? R[(size_t)s2 * n + j0 + c] : gj_zero<T>();
    }
    __syncthreads();
    T acc[TI][4];
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int i = i0 + TI * ty + ii, j = j0 + 4 * tx + jj;
            const bool inK = j >= k0 && j < k0 + b;
            acc[ii][jj] = (i < n && j < n && !inK) ? A[(size_t)i * n + j] : gj_zero<T>();
        }
    for (int s = 0; s < b; ++s) {
        T cv[TI], rv[4];
#pragma unroll
        for (int q = 0; q < TI; ++q) cv[q] = sc[TI * ty + q][s];
#pragma unroll
        for (int q = 0; q < 4; ++q) rv[q] = sr[s][4 * tx + q];
#pragma unroll
        for (int ii = 0; ii < TI; ++ii)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = gj_fms(acc[ii][jj], cv[ii], rv[jj]);
    }
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int i = i0 + TI * ty + ii, j = j0 + 4 * tx + jj;
            if (i >= n || j >= n) continue;
            // the panel's own rows take R
            A[(size_t)i * n + j] = (i >= k0 && i < k0 + b) ? sr[i - k0][4 * tx + jj] : acc[ii][jj];
        }
}

template <typename T>
static void gj_invert(T *A, T *Dinv, T *R, T *C, int n, hipStream_t s)
{
    const int b = n < kGjB ? n : kGjB, tr = 16 * gj_rows<T>();
    const dim3 gu((n + 63) / 64, (n + tr - 1) / tr), gp((n + 63) / 64, (b + 3) / 4);
    for (int k0 = 0; k0 < n; k0 += b) {
        hipLaunchKernelGGL(k_gj_diag<T>, dim3(1), dim3(256), 0, s, A, Dinv, n, k0, b);
        hipLaunchKernelGGL(k_gj_panel<T>, gp, dim3(256), 0, s, A, Dinv, R, C, n, k0, b);
        hipLaunchKernelGGL(k_gj_update<T>, gu, dim3(256), 0, s, A, R, C, n, k0, b);
    }
}

// Halves of the folded inverses, each (n/2) x (n/2) row-major, in one
// buffer: X0 even, X0 odd, X2 even, X2 odd, Re X1 even, Re X1 odd,
// Im X1 (odd -> even), Im X1 (even -> odd).
enum { kH0E = 0, kH0O, kH2E, kH2O, kH1RE, kH1RO, kH1IEO, kH1IOE, kHalves };

// Folds the full inverses X0, X2 (real) and X1 (complex) into the halves:
// for r, c < n/2 with c' = n-1-c, r' = n-1-r,
//   even = (X[r][c] + X[r][c'] + X[r'][c'] + X[r'][c]) / 4,
//   odd  = (X[r][c] - X[r][c'] + X[r'][c'] - X[r'][c]) / 4,
// and for Im X1 (J Im X1 J = -Im X1)
//   odd -> even = (I[r][c] - I[r][c'] - I[r'][c'] + I[r'][c]) / 4,
//   even -> odd = (I[r][c] + I[r][c'] - I[r'][c'] - I[r'][c]) / 4.
__global__ __launch_bounds__(256) void k_bem_fold(const double *__restrict__ X0,
                                                  const double *__restrict__ X2,
                                                  const double2 *__restrict__ X1,
                                                  double *__restrict__ Xh, int n)
{
    const int m = n >> 1;
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (r >= m || c >= m) return;
    const size_t a = (size_t)r * n + c, b = (size_t)r * n + (n - 1 - c);
    const size_t d = (size_t)(n - 1 - r) * n + (n - 1 - c), e = (size_t)(n - 1 - r) * n + c;
    const size_t o = (size_t)r * m + c, hs = (size_t)m * m;
    Xh[kH0E * hs + o] = 0.25 * ((X0[a] + X0[b]) + (X0[d] + X0[e]));
    Xh[kH0O * hs + o] = 0.25 * ((X0[a] - X0[b]) + (X0[d] - X0[e]));
    Xh[kH2E * hs + o] = 0.25 * ((X2[a] + X2[b]) + (X2[d] + X2[e]));
    Xh[kH2O * hs + o] = 0.25 * ((X2[a] - X2[b]) + (X2[d] - X2[e]));
    const double2 xa = X1[a], xb = X1[b], xd = X1[d], xe = X1[e];
    Xh[kH1RE * hs + o] = 0.25 * ((xa.x + xb.x) + (xd.x + xe.x));
    Xh[kH1RO * hs + o] = 0.25 * ((xa.x - xb.x) + (xd.x - xe.x));
    Xh[kH1IEO * hs + o] = 0.25 * ((xa.y - xb.y) - (xd.y - xe.y));
    Xh[kH1IOE * hs + o] = 0.25 * ((xa.y + xb.y) - (xd.y + xe.y));
}

// The products of the folded inverses with the split right-hand side, one
// wave per row of a half (n/2 rows per group), in the layout of bh:
//   y = 0: X0 even . e0,  1: X0 odd . o0,  2: X2 even . e2,  3: X2 odd . o2,
//   4: even part of mode 1 = Re X1 even . e1 + i Im X1 (odd -> even) . o1,
//   5: odd part of mode 1  = i Im X1 (even -> odd) . e1 + Re X1 odd . o1.
// Several right-hand sides share one read of the inverse: blockIdx.z takes
// up to NRB of them (rh.sb apart), each accumulated in the same order as a
// lone right-hand side, so every result is the same bit for bit.
constexpr int kGemvRhs = 8;

template <int NRB>
__global__ __launch_bounds__(256) void k_bem_gemv(const double *__restrict__ Xh,
                                                  const double2 *__restrict__ bh,
                                                  double2 *__restrict__ sh, int n, RhsSet rh,
                                                  int nr)
{
    const int m = n >> 1;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int which = blockIdx.y;
    const int r0 = blockIdx.z * NRB;
    if (row >= m) return;
    bool on[NRB];
#pragma unroll
    for (int c = 0; c < NRB; ++c) on[c] = r0 + c < nr && rhs_active(rh, r0 + c);
    const size_t hs = (size_t)m * m;
    double ax[NRB], ay[NRB];
#pragma unroll
    for (int c = 0; c < NRB; ++c) ax[c] = ay[c] = 0.0;
    if (which < 4) {
        const double *X = Xh + which * hs + (size_t)row * m;
        const double2 *bv = bh + which * m + r0 * rh.sb;
        for (int j = lane; j < m; j += 64) {
            const double x = X[j];
#pragma unroll
            for (int c = 0; c < NRB; ++c)
                if (on[c]) ax[c] = fma(x, bv[c * rh.sb + j].x, ax[c]);
        }
    } else {
        // which 4: Re part acts on e1, Im part (odd -> even) on o1; which 5:
        // Im part (even -> odd) on e1, Re part on o1
        const double *R = Xh + (which == 4 ? kH1RE : kH1RO) * hs + (size_t)row * m;
        const double *I = Xh + (which == 4 ? kH1IEO : kH1IOE) * hs + (size_t)row * m;
        const double2 *br = bh + 2 * n + (which == 4 ? 0 : m) + r0 * rh.sb;   // input of the Re part
        const double2 *bi = bh + 2 * n + (which == 4 ? m : 0) + r0 * rh.sb;   // input of the Im part
        for (int j = lane; j < m; j += 64) {
            const double xr = R[j], xi = I[j];
#pragma unroll
            for (int c = 0; c < NRB; ++c)
                if (on[c]) {
                    const double2 u = br[c * rh.sb + j], v = bi[c * rh.sb + j];
                    // xr u + i xi v
                    ax[c] = fma(xr, u.x, fma(-xi, v.y, ax[c]));
                    ay[c] = fma(xr, u.y, fma(xi, v.x, ay[c]));
                }
        }
    }
#pragma unroll
    for (int c = 0; c < NRB; ++c) {
        if (!on[c]) continue;
        double x = ax[c], y = ay[c];
        for (int o = 32; o > 0; o >>= 1) {
            x += __shfl_xor(x, o);
            y += __shfl_xor(y, o);
        }
        if (lane == 0) sh[(r0 + c) * rh.sb + which * m + row] = make_double2(x, y);
    }
}

// sigma (ring_sigma) and the ring charges h sigma at every node; the
// boundary-source pass computes them itself when the tree has levels >= 2
__global__ void k_bem_sigma(const double2 *__restrict__ sh, double *__restrict__ rq,
                            double *__restrict__ sig_out, int n, double h, RhsSet rh)
{
    if (!rhs_active(rh, blockIdx.z)) return;
    sh += blockIdx.z * rh.sb;
    rq += blockIdx.z * rh.sr;
    if (sig_out) sig_out += blockIdx.z * rh.sr;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= 4 * n) return;
    const int s = t / n, k = t - s * n;
    const double sg = ring_sigma(sh, s, k, n);
    rq[t] = h * sg;
    if (sig_out) sig_out[t] = sg;
}

int bem_setup(fmm_plan *pl, hipStream_t s)
{
    const int n = (int)pl->n;
    const size_t nn = (size_t)n * n;
    double2 *dinv = nullptr, *R = nullptr, *C = nullptr;
    const int b = n < kGjB ? n : kGjB;
    FMM_HIP(pl, hipMalloc(&pl->X0, nn * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->X2, nn * sizeof(double)));
    FMM_HIP(pl, hipMalloc(&pl->X1, nn * sizeof(double2)));
    FMM_HIP(pl, hipMalloc(&dinv, (size_t)b * b * sizeof(double2)));
    FMM_HIP(pl, hipMalloc(&R, (size_t)b * n * sizeof(double2)));
    FMM_HIP(pl, hipMalloc(&C, (size_t)b * n * sizeof(double2)));
    const dim3 g2((n + 63) / 64, (n + 3) / 4);
    hipLaunchKernelGGL(k_bem_build, g2, dim3(256), 0, s, pl->X0, pl->X2, pl->X1, n);
    // the real blocks, then the complex one
    gj_invert<double>(pl->X0, reinterpret_cast<double *>(dinv), reinterpret_cast<double *>(R),
                      reinterpret_cast<double *>(C), n, s);
    gj_invert<double>(pl->X2, reinterpret_cast<double *>(dinv), reinterpret_cast<double *>(R),
                      reinterpret_cast<double *>(C), n, s);
    static_assert(sizeof(gj_c) == sizeof(double2), "complex layout");
    gj_invert<gj_c>(reinterpret_cast<gj_c *>(pl->X1), reinterpret_cast<gj_c *>(dinv),
                    reinterpret_cast<gj_c *>(R), reinterpret_cast<gj_c *>(C), n, s);
    // fold into the even/odd halves and keep only those
    FMM_HIP(pl, hipMalloc(&pl->Xh, (size_t)kHalves * (nn / 4) * sizeof(double)));
    hipLaunchKernelGGL(k_bem_fold, dim3((n / 2 + 63) / 64, (n / 2 + 3) / 4), dim3(256), 0, s,
                       pl->X0, pl->X2, pl->X1, pl->Xh, n);
    FMM_HIP(pl, hipGetLastError());
    FMM_HIP(pl, hipStreamSynchronize(s));
    FMM_HIP(pl, hipFree(dinv));
    FMM_HIP(pl, hipFree(R));
    FMM_HIP(pl, hipFree(C));
    FMM_HIP(pl, hipFree(pl->X0));
    FMM_HIP(pl, hipFree(pl->X2));
    FMM_HIP(pl, hipFree(pl->X1));
    pl->X0 = pl->X2 = nullptr;
    pl->X1 = nullptr;
    return FMM_OK;
}

// sigma = -S^{-1} phi_ring: the products of the folded inverses with the
// split right-hand side pl->bhat (written by the ring-target kernel of the
// volume pass) into pl->shat.  With levels >= 2 the boundary-source pass
// forms sigma and the charges from pl->shat inside its P2M; otherwise they
// are formed here (pl->ring_q, and sigma_out when given).
int bem_apply(fmm_plan *pl, double *sigma_out, const RhsSet &rh, int nr, hipStream_t s)
{
    const int n = (int)pl->n;
    StageTimer t(pl, FMM_STAGE_BEM, s);
    const int m = n / 2;
    if (nr == 1)
        hipLaunchKernelGGL(k_bem_gemv<1>, dim3((m + 3) / 4, 6, 1), dim3(256), 0, s, pl->Xh, pl->bhat,
                           pl->shat, n, rh, nr);
    else
        hipLaunchKernelGGL(k_bem_gemv<kGemvRhs>, dim3((m + 3) / 4, 6, (nr + kGemvRhs - 1) / kGemvRhs),
                           dim3(256), 0, s, pl->Xh, pl->bhat, pl->shat, n, rh, nr);
    if (pl->L < 2)
        hipLaunchKernelGGL(k_bem_sigma, dim3((4 * n + 255) / 256, 1, nr), dim3(256), 0, s, pl->shat,
                           pl->ring_q, sigma_out, n, pl->h, rh);
    FMM_HIP(pl, hipGetLastError());
    return FMM_OK;
}

}  // namespace fmmprec
