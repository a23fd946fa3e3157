/*
 * fmm_oracle.c -- plain, slow, obviously correct CPU FP64 reference for the
 * FMM-preconditioned Krylov solve of the 5-point Poisson matrix
 * (Ibeid, Yokota, Pestana, Keyes, "Fast Multipole Preconditioners for Sparse
 * Matrices Arising from Elliptic Equations", arXiv:1308.3339).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  The product library never links,
 * includes or calls anything from this directory, and this file includes
 * nothing from the product.
 *
 * Everything is double precision, double complex for the expansions, libm
 * log/sqrt, no SIMD intrinsics, no blocking.  OpenMP is used only over
 * independent targets / independent cells (each writes its own output).
 *
 * Readings of the paper implemented here (the GPU library implements the
 * same readings independently):
 *   - Kernel G(r) = -(1/2pi) log r (Sec. 4.2 eq. for G; Sec. 5.3).  The
 *     expansions accumulate sum_j q_j log(z - z_j); the factor -1/(2pi) is
 *     applied once, after near and far field are added.
 *   - A coincident source/target pair (r == 0) contributes q * self_log in
 *     log-space instead of q * log r.  For grid problems self_log =
 *     log(eps_s h) regularises only the singular self term (the smoothed
 *     kernel of Sec. 4.2 read as a self-cell value); for point clouds
 *     self_log = 0 drops the i == j term.
 *   - p counts coefficients: M_0..M_{p-1}, L_0..L_{p-1} (Sec. 5.3).
 *   - Uniform quadtree with L levels below the root; a point belongs to leaf
 *     min(max(floor((x - x0)/side * 2^L), 0), 2^L - 1) per axis.  Expansion
 *     centres are geometric cell centres.
 *   - Interaction list (Sec. 5.2, the Greengard-Rokhlin rule): children of
 *     the parent's 3x3 neighbourhood that are not adjacent (edge or corner)
 *     to the target cell, at levels 2..L.  Near field: the 3x3 leaves around
 *     the target's leaf, self leaf included.
 *   - With a MAC theta (Sec. 5.2, dual tree traversal): a cell pair of one
 *     level is well separated when the two cell radii (half diagonals) sum
 *     to less than theta times the centre distance; pairs that fail are
 *     split together, leaf pairs that fail are P2P.
 *   - Operators P2M, M2M, M2L, L2L, L2P exactly as listed in Sec. 5.3
 *     (items 1-5), unscaled, powers by repeated multiplication.
 *   - Boundary correction (Sec. 4.1, eqs. ubound/uinter with zero Dirichlet
 *     data): collocation at the 4n ring nodes, constant elements of length h,
 *     analytic self panel; sigma = -S^{-1} phi_ring; z = phi + sum h sigma G.
 *   - Krylov: right-preconditioned FGMRES(m) with modified Gram-Schmidt and
 *     Givens rotations (the paper cites GMRES, Sec. 1), x0 given, stop when
 *     the true residual ||b - Ax|| / ||b|| <= tol.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ======================================================================== */
/* small helpers                                                            */
/* ======================================================================== */

/* binomial coefficient C(a, b); exact in double for the orders used here */
static double binom(int a, int b)
{
    if (b < 0 || b > a) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= b; ++i) r = r * (double)(a - b + i) / (double)i;
    return floor(r + 0.5);
}

/* z^k by repeated multiplication (k >= 0) */
static cplx cpow_int(cplx z, int k)
{
    cplx r = 1.0;
    for (int i = 0; i < k; ++i) r *= z;
    return r;
}

static void unpack(int p, const double *a, cplx *z)
{
    for (int n = 0; n < p; ++n) z[n] = a[2 * n] + I * a[2 * n + 1];
}

static void pack(int p, const cplx *z, double *a)
{
    for (int n = 0; n < p; ++n) { a[2 * n] = creal(z[n]); a[2 * n + 1] = cimag(z[n]); }
}

/* ======================================================================== */
/* Sec. 5.3: the five translation operators                                 */
/* ======================================================================== */

/* Item 1, P2M:  M_0 = sum f_j,  M_n = sum -f_j (-z_{mu j})^n / n.
 * -z_{mu j} = z_j - z_mu is the source position relative to the centre. */
static void p2m_c(int p, cplx centre, int ns, const double *sx, const double *sy,
                  const double *sq, const int *idx, cplx *M)
{
    for (int a = 0; a < ns; ++a) {
        int j = idx ? idx[a] : a;
        cplx s = (sx[j] + I * sy[j]) - centre;
        M[0] += sq[j];
        for (int n = 1; n < p; ++n)
            M[n] += -sq[j] * cpow_int(s, n) / (double)n;
    }
}

/* Item 2, M2M:  M_0(M) = M_0(mu),
 * M_n(M) = -M_0(mu) (-z_{M mu})^n / n + sum_{k=1..n} M_k(mu) (-z_{M mu})^{n-k} C(n-1, k-1).
 * c = -z_{M mu} = z_mu - z_M (child centre minus parent centre).  Adds into Mp. */
static void m2m_c(int p, const cplx *Mc, cplx c, cplx *Mp)
{
    Mp[0] += Mc[0];
    for (int n = 1; n < p; ++n) {
        cplx acc = -Mc[0] * cpow_int(c, n) / (double)n;
        for (int k = 1; k <= n; ++k)
            acc += Mc[k] * cpow_int(c, n - k) * binom(n - 1, k - 1);
        Mp[n] += acc;
    }
}

/* Item 3, M2L:  d = z_{Lambda M} = z_Lambda - z_M (target centre minus source centre).
 * L_0 += M_0 log(d) + sum_{k=1..p-1} M_k / d^k
 * L_n += -M_0 / ((-d)^n n) + sum_{k=1..p-1} (-1)^n M_k C(n+k-1, k-1) / d^{n+k}.
 * Principal branch of the complex log; only Re L_0 ever reaches a potential. */
static void m2l_c(int p, const cplx *M, cplx d, cplx *L)
{
    cplx acc0 = M[0] * clog(d);
    for (int k = 1; k < p; ++k) acc0 += M[k] / cpow_int(d, k);
    L[0] += acc0;
    for (int n = 1; n < p; ++n) {
        cplx acc = -M[0] / (cpow_int(-d, n) * (double)n);
        double sgn = (n % 2 == 0) ? 1.0 : -1.0;
        for (int k = 1; k < p; ++k)
            acc += sgn * M[k] * binom(n + k - 1, k - 1) / cpow_int(d, n + k);
        L[n] += acc;
    }
}

/* Item 4, L2L:  c = z_{lambda Lambda} = z_lambda - z_Lambda (child minus parent).
 * L_n(lambda) = sum_{k=n..p-1} L_k(Lambda) c^{k-n} C(k, n).  Adds into Lc. */
static void l2l_c(int p, const cplx *Lp, cplx c, cplx *Lc)
{
    for (int n = 0; n < p; ++n) {
        cplx acc = 0.0;
        for (int k = n; k < p; ++k) acc += Lp[k] * cpow_int(c, k - n) * binom(k, n);
        Lc[n] += acc;
    }
}

/* Item 5, L2P:  u_i = Re sum_n L_n z_{i lambda}^n, z_{i lambda} = z_i - z_lambda. */
static double l2p_c(int p, const cplx *L, cplx t)
{
    cplx acc = 0.0;
    for (int n = 0; n < p; ++n) acc += L[n] * cpow_int(t, n);
    return creal(acc);
}

/* Evaluation of a multipole expansion at w = z - z_centre (used only by tests):
 * Re( M_0 log w + sum_{n>=1} M_n / w^n ).  This is the series that P2M truncates. */
static double m2p_c(int p, const cplx *M, cplx w)
{
    cplx acc = M[0] * clog(w);
    for (int n = 1; n < p; ++n) acc += M[n] / cpow_int(w, n);
    return creal(acc);
}

/* ---- exported single-operator entry points (complex arrays as re/im pairs) */
void orc_p2m(int p, double cx, double cy, int ns, const double *sx,
             const double *sy, const double *sq, double *Mout)
{
    cplx *M = (cplx *)calloc((size_t)p, sizeof(cplx));
    p2m_c(p, cx + I * cy, ns, sx, sy, sq, NULL, M);
    pack(p, M, Mout);
    free(M);
}

void orc_m2m(int p, const double *Mc_in, double cx, double cy, double *Mp_out)
{
    cplx *Mc = (cplx *)calloc((size_t)p, sizeof(cplx));
    cplx *Mp = (cplx *)calloc((size_t)p, sizeof(cplx));
    unpack(p, Mc_in, Mc);
    m2m_c(p, Mc, cx + I * cy, Mp);
    pack(p, Mp, Mp_out);
    free(Mc); free(Mp);
}

void orc_m2l(int p, const double *M_in, double dx, double dy, double *L_out)
{
    cplx *M = (cplx *)calloc((size_t)p, sizeof(cplx));
    cplx *L = (cplx *)calloc((size_t)p, sizeof(cplx));
    unpack(p, M_in, M);
    m2l_c(p, M, dx + I * dy, L);
    pack(p, L, L_out);
    free(M); free(L);
}

void orc_l2l(int p, const double *Lp_in, double cx, double cy, double *Lc_out)
{
    cplx *Lp = (cplx *)calloc((size_t)p, sizeof(cplx));
    cplx *Lc = (cplx *)calloc((size_t)p, sizeof(cplx));
    unpack(p, Lp_in, Lp);
    l2l_c(p, Lp, cx + I * cy, Lc);
    pack(p, Lc, Lc_out);
    free(Lp); free(Lc);
}

double orc_l2p(int p, const double *L_in, double tx, double ty)
{
    cplx *L = (cplx *)calloc((size_t)p, sizeof(cplx));
    unpack(p, L_in, L);
    double r = l2p_c(p, L, tx + I * ty);
    free(L);
    return r;
}

double orc_m2p(int p, const double *M_in, double wx, double wy)
{
    cplx *M = (cplx *)calloc((size_t)p, sizeof(cplx));
    unpack(p, M_in, M);
    double r = m2p_c(p, M, wx + I * wy);
    free(M);
    return r;
}

/* ======================================================================== */
/* Direct sum (Sec. 5.1 eq. volume_integral): the exact reference.            */
/* u_t = -(1/2pi) sum_j q_j k(r_tj),  k(r) = log r for r > 0, self_log for r == 0 */
/* ======================================================================== */
void orc_direct(int ns, const double *sx, const double *sy, const double *sq,
                int nt, const double *tx, const double *ty, double self_log,
                double *u)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < nt; ++t) {
        double acc = 0.0;
        for (int j = 0; j < ns; ++j) {
            double dx = tx[t] - sx[j], dy = ty[t] - sy[j];
            double r = sqrt(dx * dx + dy * dy);
            acc += sq[j] * (r == 0.0 ? self_log : log(r));
        }
        u[t] = -acc / (2.0 * ORC_PI);
    }
}

/* ======================================================================== */
/* Uniform quadtree and interaction lists (Sec. 5.1, 5.2)                    */
/* ======================================================================== */

static int leaf_coord(double v, double v0, double side, int nl)
{
    double f = floor((v - v0) / side * (double)nl);
    if (f < 0.0) f = 0.0;
    if (f > (double)(nl - 1)) f = (double)(nl - 1);
    return (int)f;
}

/* Morton index of leaf (lx, ly) at level L: bit b of lx goes to bit 2b and
 * bit b of ly to bit 2b + 1 (x bits in the even positions). */
static int64_t morton_of(int lx, int ly, int L)
{
    int64_t m = 0;
    for (int b = 0; b < L; ++b) {
        m |= (int64_t)((lx >> b) & 1) << (2 * b);
        m |= (int64_t)((ly >> b) & 1) << (2 * b + 1);
    }
    return m;
}

/* Points bucketed by leaf (Sec. 5.1 tree construction on the uniform tree):
 * a stable counting sort by leaf key, key = row-major index ly * 2^L + lx
 * (order 0) or the Morton index (order 1).  scount (4^L + 1) receives the
 * first sorted position of each key and sorder (ns) the original index of
 * each sorted position; points of one leaf keep their original order. */
int orc_bucket_points(int L, double x0, double y0, double side, int order, int ns,
                      const double *sx, const double *sy, int *scount, int *sorder)
{
    if (L < 0 || L > 15 || ns < 0 || (order != 0 && order != 1)) return -1;
    int nl = 1 << L;
    int64_t nleaf = (int64_t)nl * nl;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    int64_t *fill = (int64_t *)calloc((size_t)nleaf, sizeof(int64_t));
    for (int64_t c = 0; c <= nleaf; ++c) scount[c] = 0;
    for (int j = 0; j < ns; ++j) {
        int lx = leaf_coord(sx[j], x0, side, nl), ly = leaf_coord(sy[j], y0, side, nl);
        key[j] = order ? morton_of(lx, ly, L) : (int64_t)ly * nl + lx;
        scount[key[j] + 1]++;
    }
    for (int64_t c = 0; c < nleaf; ++c) scount[c + 1] += scount[c];
    for (int j = 0; j < ns; ++j) sorder[scount[key[j]] + fill[key[j]]++] = j;
    free(key);
    free(fill);
    return 0;
}

/* Fills up to 27 (sx, sy) pairs of the M2L list of cell (ix, iy) at level l;
 * returns the count.  Cells outside [0, 2^l)^2 do not exist. */
int orc_m2l_list(int l, int ix, int iy, int *out)
{
    int ncell = 1 << l, cnt = 0;
    if (l < 2) return 0;
    int px = ix / 2, py = iy / 2, npar = ncell / 2;
    for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) {
            int qx = px + a, qy = py + b;
            if (qx < 0 || qy < 0 || qx >= npar || qy >= npar) continue;
            for (int d = 0; d < 2; ++d)
                for (int c = 0; c < 2; ++c) {
                    int sx = 2 * qx + c, sy = 2 * qy + d;
                    if (abs(sx - ix) <= 1 && abs(sy - iy) <= 1) continue; /* adjacent */
                    out[2 * cnt] = sx; out[2 * cnt + 1] = sy; ++cnt;
                }
        }
    return cnt;
}

/* ======================================================================== */
/* The FMM (Sec. 5): sources and targets attached to leaves of a uniform    */
/* tree over the square [x0, x0+side] x [y0, y0+side] with L levels.          */
/* ======================================================================== */
static cplx cell_centre(int l, int ix, int iy, double x0, double y0, double side)
{
    double w = side / (double)(1 << l);
    return (x0 + (ix + 0.5) * w) + I * (y0 + (iy + 0.5) * w);
}

int orc_fmm(int L, double x0, double y0, double side, int p,
            int ns, const double *sx, const double *sy, const double *sq,
            int nt, const double *tx, const double *ty, double self_log,
            double *u)
{
    if (L < 0 || p < 1) return -1;
    int nl = 1 << L, nleaf = nl * nl;

    /* bucket the sources by leaf (counting sort, stable) */
    int *scount = (int *)calloc((size_t)nleaf + 1, sizeof(int));
    int *sleaf = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
    for (int j = 0; j < ns; ++j) {
        int lx = leaf_coord(sx[j], x0, side, nl), ly = leaf_coord(sy[j], y0, side, nl);
        sleaf[j] = ly * nl + lx;
        scount[sleaf[j] + 1]++;
    }
    for (int c = 0; c < nleaf; ++c) scount[c + 1] += scount[c];
    int *sorder = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
    int *fill = (int *)calloc((size_t)nleaf, sizeof(int));
    for (int j = 0; j < ns; ++j) sorder[scount[sleaf[j]] + fill[sleaf[j]]++] = j;
    free(fill);

    /* expansions per level: level l has 4^l cells, row-major (iy * 2^l + ix) */
    cplx **M = (cplx **)calloc((size_t)L + 1, sizeof(cplx *));
    cplx **Lx = (cplx **)calloc((size_t)L + 1, sizeof(cplx *));
    for (int l = 0; l <= L; ++l) {
        size_t nc = (size_t)1 << (2 * l);
        M[l] = (cplx *)calloc(nc * (size_t)p, sizeof(cplx));
        Lx[l] = (cplx *)calloc(nc * (size_t)p, sizeof(cplx));
    }

    /* P2M at the leaves */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nleaf; ++c) {
        cplx ctr = cell_centre(L, c % nl, c / nl, x0, y0, side);
        p2m_c(p, ctr, scount[c + 1] - scount[c], sx, sy, sq, sorder + scount[c],
              M[L] + (size_t)c * p);
    }

    /* M2M from level l+1 to level l (only levels >= 2 are ever used) */
    for (int l = L - 1; l >= 2; --l) {
        int nc = 1 << l;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc * nc; ++c) {
            int ix = c % nc, iy = c / nc;
            cplx pc = cell_centre(l, ix, iy, x0, y0, side);
            for (int d = 0; d < 2; ++d)
                for (int e = 0; e < 2; ++e) {
                    int cx = 2 * ix + e, cy = 2 * iy + d;
                    cplx cc = cell_centre(l + 1, cx, cy, x0, y0, side);
                    m2m_c(p, M[l + 1] + ((size_t)cy * (2 * nc) + cx) * p, cc - pc,
                          M[l] + (size_t)c * p);
                }
        }
    }

    /* M2L at levels 2..L, then L2L to the next level */
    for (int l = 2; l <= L; ++l) {
        int nc = 1 << l;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc * nc; ++c) {
            int ix = c % nc, iy = c / nc, list[54];
            cplx tc = cell_centre(l, ix, iy, x0, y0, side);
            int cnt = orc_m2l_list(l, ix, iy, list);
            for (int a = 0; a < cnt; ++a) {
                int sxc = list[2 * a], syc = list[2 * a + 1];
                cplx scc = cell_centre(l, sxc, syc, x0, y0, side);
                m2l_c(p, M[l] + ((size_t)syc * nc + sxc) * p, tc - scc,
                      Lx[l] + (size_t)c * p);
            }
        }
        if (l < L) {
            int nch = 2 * nc;
#pragma omp parallel for schedule(static)
            for (int c = 0; c < nch * nch; ++c) {
                int cx = c % nch, cy = c / nch;
                cplx cc = cell_centre(l + 1, cx, cy, x0, y0, side);
                cplx pc = cell_centre(l, cx / 2, cy / 2, x0, y0, side);
                l2l_c(p, Lx[l] + ((size_t)(cy / 2) * nc + cx / 2) * p, cc - pc,
                      Lx[l + 1] + (size_t)c * p);
            }
        }
    }

    /* L2P + P2P for every target, from the leaf it is attached to */
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < nt; ++t) {
        int lx = leaf_coord(tx[t], x0, side, nl), ly = leaf_coord(ty[t], y0, side, nl);
        cplx tz = tx[t] + I * ty[t];
        double far = 0.0;
        if (L >= 2) {
            cplx ctr = cell_centre(L, lx, ly, x0, y0, side);
            far = l2p_c(p, Lx[L] + ((size_t)ly * nl + lx) * p, tz - ctr);
        }
        double near = 0.0;
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
                int qx = lx + a, qy = ly + b;
                if (qx < 0 || qy < 0 || qx >= nl || qy >= nl) continue;
                int c = qy * nl + qx;
                for (int s = scount[c]; s < scount[c + 1]; ++s) {
                    int j = sorder[s];
                    double dx = tx[t] - sx[j], dy = ty[t] - sy[j];
                    double r = sqrt(dx * dx + dy * dy);
                    near += sq[j] * (r == 0.0 ? self_log : log(r));
                }
            }
        u[t] = -(far + near) / (2.0 * ORC_PI);
    }

    for (int l = 0; l <= L; ++l) { free(M[l]); free(Lx[l]); }
    free(M); free(Lx); free(scount); free(sleaf); free(sorder);
    return 0;
}

/* ======================================================================== */
/* Dual tree traversal with a multipole acceptance criterion (Sec. 5.2).     */
/* Target and source trees are the same uniform quadtree.  A pair of cells  */
/* (A, B) of one level is well separated when r_A + r_B < theta |c_A - c_B|, */
/* r the cell radius (half the diagonal), c the geometric centres; such a   */
/* pair is one M2L.  A pair that fails the test is one P2P pair if both     */
/* cells are leaves; otherwise both cells are split (they have the same     */
/* size on a uniform tree, so the rule "split the larger cell" ties and     */
/* both are split) and the traversal recurses on the 16 child pairs.  It    */
/* starts at (root, root).  theta in (0, 1]; theta in (1/sqrt2, 1] gives    */
/* back the interaction lists above.                                        */
/* ======================================================================== */
typedef struct { int l, t, s; } orc_pair;   /* level, target cell, source cell (row-major) */
typedef struct { orc_pair *v; size_t n, cap; } orc_pairs;

static void pairs_push(orc_pairs *a, int l, int t, int s)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 1024;
        a->v = (orc_pair *)realloc(a->v, a->cap * sizeof(orc_pair));
    }
    a->v[a->n].l = l; a->v[a->n].t = t; a->v[a->n].s = s;
    a->n++;
}

typedef struct { int L; double side, theta; orc_pairs m2l, p2p; } dtt_ctx;

static void dtt_visit(dtt_ctx *c, int l, int ax, int ay, int bx, int by)
{
    int nc = 1 << l;
    double w = c->side / (double)nc;
    double r = 0.5 * sqrt(2.0) * w;
    double dx = (double)(ax - bx) * w, dy = (double)(ay - by) * w;
    if (r + r < c->theta * sqrt(dx * dx + dy * dy)) {
        pairs_push(&c->m2l, l, ay * nc + ax, by * nc + bx);
        return;
    }
    if (l == c->L) {
        pairs_push(&c->p2p, l, ay * nc + ax, by * nc + bx);
        return;
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            dtt_visit(c, l + 1, 2 * ax + (a & 1), 2 * ay + (a >> 1), 2 * bx + (b & 1),
                      2 * by + (b >> 1));
}

static int dtt_run(int L, double side, double theta, dtt_ctx *c)
{
    if (L < 0 || !(theta > 0.0) || theta > 1.0) return -1;
    memset(c, 0, sizeof(*c));
    c->L = L; c->side = side; c->theta = theta;
    dtt_visit(c, 0, 0, 0, 0, 0);
    return 0;
}

/* Interaction pairs of the traversal on a tree with L levels (unit root;
 * the lists do not depend on the root's size).  counts[0] = M2L pairs,
 * counts[1] = P2P leaf pairs.  When m2l / p2p are not null they receive
 * (level, target cell, source cell) triples and (target leaf, source leaf)
 * pairs, in traversal order. */
int orc_dtt_lists(int L, double theta, int64_t *counts, int *m2l, int *p2p)
{
    dtt_ctx c;
    if (dtt_run(L, 1.0, theta, &c) != 0) return -1;
    counts[0] = (int64_t)c.m2l.n;
    counts[1] = (int64_t)c.p2p.n;
    for (size_t i = 0; m2l && i < c.m2l.n; ++i) {
        m2l[3 * i] = c.m2l.v[i].l; m2l[3 * i + 1] = c.m2l.v[i].t; m2l[3 * i + 2] = c.m2l.v[i].s;
    }
    for (size_t i = 0; p2p && i < c.p2p.n; ++i) {
        p2p[2 * i] = c.p2p.v[i].t; p2p[2 * i + 1] = c.p2p.v[i].s;
    }
    free(c.m2l.v); free(c.p2p.v);
    return 0;
}

/* pairs grouped by target: start[t] .. start[t+1] index src[] (stable) */
static void group_by_target(const orc_pairs *a, int level, int ncell, int **start, int **src)
{
    int *st = (int *)calloc((size_t)ncell + 1, sizeof(int));
    for (size_t i = 0; i < a->n; ++i)
        if (a->v[i].l == level) st[a->v[i].t + 1]++;
    for (int t = 0; t < ncell; ++t) st[t + 1] += st[t];
    int *sr = (int *)malloc(sizeof(int) * (size_t)(st[ncell] > 0 ? st[ncell] : 1));
    int *fill = (int *)calloc((size_t)ncell, sizeof(int));
    for (size_t i = 0; i < a->n; ++i)
        if (a->v[i].l == level) sr[st[a->v[i].t] + fill[a->v[i].t]++] = a->v[i].s;
    free(fill);
    *start = st;
    *src = sr;
}

/* The FMM of orc_fmm with the interactions of the dual tree traversal:
 * P2M at the leaves, M2M up to the root, the traversal's M2L pairs at every
 * level, L2L down, L2P at the targets' leaves, and the traversal's P2P leaf
 * pairs for the near field. */
int orc_fmm_theta(int L, double x0, double y0, double side, int p, double theta,
                  int ns, const double *sx, const double *sy, const double *sq,
                  int nt, const double *tx, const double *ty, double self_log,
                  double *u)
{
    if (L < 0 || p < 1) return -1;
    dtt_ctx c;
    if (dtt_run(L, side, theta, &c) != 0) return -1;
    int nl = 1 << L, nleaf = nl * nl;

    int *scount = (int *)calloc((size_t)nleaf + 1, sizeof(int));
    int *sleaf = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
    for (int j = 0; j < ns; ++j) {
        int lx = leaf_coord(sx[j], x0, side, nl), ly = leaf_coord(sy[j], y0, side, nl);
        sleaf[j] = ly * nl + lx;
        scount[sleaf[j] + 1]++;
    }
    for (int k = 0; k < nleaf; ++k) scount[k + 1] += scount[k];
    int *sorder = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
    int *fill = (int *)calloc((size_t)nleaf, sizeof(int));
    for (int j = 0; j < ns; ++j) sorder[scount[sleaf[j]] + fill[sleaf[j]]++] = j;
    free(fill);

    cplx **M = (cplx **)calloc((size_t)L + 1, sizeof(cplx *));
    cplx **Lx = (cplx **)calloc((size_t)L + 1, sizeof(cplx *));
    for (int l = 0; l <= L; ++l) {
        size_t nc = (size_t)1 << (2 * l);
        M[l] = (cplx *)calloc(nc * (size_t)p, sizeof(cplx));
        Lx[l] = (cplx *)calloc(nc * (size_t)p, sizeof(cplx));
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nleaf; ++k) {
        cplx ctr = cell_centre(L, k % nl, k / nl, x0, y0, side);
        p2m_c(p, ctr, scount[k + 1] - scount[k], sx, sy, sq, sorder + scount[k],
              M[L] + (size_t)k * p);
    }
    for (int l = L - 1; l >= 0; --l) {
        int nc = 1 << l;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nc * nc; ++k) {
            int ix = k % nc, iy = k / nc;
            cplx pc = cell_centre(l, ix, iy, x0, y0, side);
            for (int d = 0; d < 2; ++d)
                for (int e = 0; e < 2; ++e) {
                    int cx = 2 * ix + e, cy = 2 * iy + d;
                    cplx cc = cell_centre(l + 1, cx, cy, x0, y0, side);
                    m2m_c(p, M[l + 1] + ((size_t)cy * (2 * nc) + cx) * p, cc - pc,
                          M[l] + (size_t)k * p);
                }
        }
    }
    for (int l = 0; l <= L; ++l) {
        int nc = 1 << l, *st, *sr;
        group_by_target(&c.m2l, l, nc * nc, &st, &sr);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nc * nc; ++k) {
            cplx tc = cell_centre(l, k % nc, k / nc, x0, y0, side);
            for (int a = st[k]; a < st[k + 1]; ++a) {
                int s = sr[a];
                cplx scc = cell_centre(l, s % nc, s / nc, x0, y0, side);
                m2l_c(p, M[l] + (size_t)s * p, tc - scc, Lx[l] + (size_t)k * p);
            }
        }
        free(st); free(sr);
        if (l < L) {
            int nch = 2 * nc;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nch * nch; ++k) {
                int cx = k % nch, cy = k / nch;
                cplx cc = cell_centre(l + 1, cx, cy, x0, y0, side);
                cplx pc = cell_centre(l, cx / 2, cy / 2, x0, y0, side);
                l2l_c(p, Lx[l] + ((size_t)(cy / 2) * nc + cx / 2) * p, cc - pc,
                      Lx[l + 1] + (size_t)k * p);
            }
        }
    }
    int *nst, *nsr;
    group_by_target(&c.p2p, L, nleaf, &nst, &nsr);
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < nt; ++t) {
        int lx = leaf_coord(tx[t], x0, side, nl), ly = leaf_coord(ty[t], y0, side, nl);
        int tl = ly * nl + lx;
        cplx tz = tx[t] + I * ty[t];
        double far = l2p_c(p, Lx[L] + (size_t)tl * p, tz - cell_centre(L, lx, ly, x0, y0, side));
        double near = 0.0;
        for (int a = nst[tl]; a < nst[tl + 1]; ++a) {
            int sl = nsr[a];
            for (int s = scount[sl]; s < scount[sl + 1]; ++s) {
                int j = sorder[s];
                double dx = tx[t] - sx[j], dy = ty[t] - sy[j];
                double r = sqrt(dx * dx + dy * dy);
                near += sq[j] * (r == 0.0 ? self_log : log(r));
            }
        }
        u[t] = -(far + near) / (2.0 * ORC_PI);
    }
    for (int l = 0; l <= L; ++l) { free(M[l]); free(Lx[l]); }
    free(M); free(Lx); free(scount); free(sleaf); free(sorder); free(nst); free(nsr);
    free(c.m2l.v); free(c.p2p.v);
    return 0;
}

/* ======================================================================== */
/* Grid problem: 5-point FD Poisson on the unit square, zero Dirichlet data */
/* interior node (i, j), i, j = 0..n-1 sits at ((i+1)h, (j+1)h), h = 1/(n+1), */
/* stored row-major at j*n + i.                                              */
/* ======================================================================== */

/* w = A v, (Av)_ij = (4 v_ij - v_{i-1,j} - v_{i+1,j} - v_{i,j-1} - v_{i,j+1}) / h^2 */
void orc_stencil(int n, const double *v, double *w)
{
    double h = 1.0 / (double)(n + 1), ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double c = 4.0 * v[(size_t)j * n + i];
            if (i > 0) c -= v[(size_t)j * n + i - 1];
            if (i < n - 1) c -= v[(size_t)j * n + i + 1];
            if (j > 0) c -= v[(size_t)(j - 1) * n + i];
            if (j < n - 1) c -= v[(size_t)(j + 1) * n + i];
            w[(size_t)j * n + i] = c * ih2;
        }
}

void orc_grid_points(int n, double *x, double *y)
{
    double h = 1.0 / (double)(n + 1);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            x[(size_t)j * n + i] = (double)(i + 1) * h;
            y[(size_t)j * n + i] = (double)(j + 1) * h;
        }
}

/* The 4n Dirichlet nodes the stencil touches (corners excluded), counter-
 * clockwise: bottom ((k+1)h, 0), right (1, (k+1)h), top ((n-k)h, 1),
 * left (0, (n-k)h), k = 0..n-1.  Node s*n + k. */
void orc_ring_points(int n, double *x, double *y)
{
    double h = 1.0 / (double)(n + 1);
    for (int k = 0; k < n; ++k) {
        x[k] = (k + 1) * h;          y[k] = 0.0;
        x[n + k] = 1.0;              y[n + k] = (k + 1) * h;
        x[2 * n + k] = (n - k) * h;  y[2 * n + k] = 1.0;
        x[3 * n + k] = 0.0;          y[3 * n + k] = (n - k) * h;
    }
}

/* Sec. 4.3 boundary matrix, collocation with constant elements of length h
 * centred on the ring nodes: S_kl = h G(|y_k - y_l|) for k != l and the exact
 * panel integral S_kk = int_{-h/2}^{h/2} G(|t|) dt = -(h/2pi)(log(h/2) - 1). */
void orc_bem_matrix(int n, double *S)
{
    int m = 4 * n;
    double h = 1.0 / (double)(n + 1);
    double *x = (double *)malloc(sizeof(double) * m), *y = (double *)malloc(sizeof(double) * m);
    orc_ring_points(n, x, y);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) {
            if (k == l) {
                S[(size_t)k * m + l] = -(h / (2.0 * ORC_PI)) * (log(h / 2.0) - 1.0);
            } else {
                double dx = x[k] - x[l], dy = y[k] - y[l];
                S[(size_t)k * m + l] = -h * log(sqrt(dx * dx + dy * dy)) / (2.0 * ORC_PI);
            }
        }
    free(x); free(y);
}

/* Dense LU with partial pivoting, in place, row-major m x m. */
int orc_lu_factor(int m, double *A, int *piv)
{
    for (int k = 0; k < m; ++k) {
        int pr = k;
        double best = fabs(A[(size_t)k * m + k]);
        for (int i = k + 1; i < m; ++i)
            if (fabs(A[(size_t)i * m + k]) > best) { best = fabs(A[(size_t)i * m + k]); pr = i; }
        piv[k] = pr;
        if (best == 0.0) return -1;
        if (pr != k)
            for (int c = 0; c < m; ++c) {
                double t = A[(size_t)k * m + c];
                A[(size_t)k * m + c] = A[(size_t)pr * m + c];
                A[(size_t)pr * m + c] = t;
            }
        double d = A[(size_t)k * m + k];
#pragma omp parallel for schedule(static)
        for (int i = k + 1; i < m; ++i) {
            double f = A[(size_t)i * m + k] / d;
            A[(size_t)i * m + k] = f;
            for (int c = k + 1; c < m; ++c) A[(size_t)i * m + c] -= f * A[(size_t)k * m + c];
        }
    }
    return 0;
}

void orc_lu_solve(int m, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < m; ++k)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < m; ++i) {
        double s = b[i];
        for (int c = 0; c < i; ++c) s -= LU[(size_t)i * m + c] * b[c];
        b[i] = s;
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = b[i];
        for (int c = i + 1; c < m; ++c) s -= LU[(size_t)i * m + c] * b[c];
        b[i] = s / LU[(size_t)i * m + i];
    }
}

/* ======================================================================== */
/* The FMM-BEM preconditioner z = P^{-1} r (Sec. 3.3, Fig. 1; Sec. 4.1)      */
/* ======================================================================== */
typedef struct {
    int n, p, bem, exact, L;
    double h, self_log;
    double theta;      /* 0: interaction lists; else the traversal's MAC */
    double *gx, *gy;   /* interior nodes   */
    double *rx, *ry;   /* ring nodes (4n)  */
    double *LU;        /* factored S       */
    int *piv;
    double *tx, *ty;   /* pass-1 targets: interior then ring */
} orc_pc;

void *orc_pc_create(int n, int p, double eps_s, int bem, int exact, double theta)
{
    if (n < 8 || (n & (n - 1)) != 0) return NULL;
    if (theta < 0.0 || theta > 1.0) return NULL;
    orc_pc *pc = (orc_pc *)calloc(1, sizeof(orc_pc));
    pc->theta = theta;
    size_t N = (size_t)n * n;
    int m = 4 * n;
    pc->n = n; pc->p = p; pc->bem = bem; pc->exact = exact;
    pc->h = 1.0 / (double)(n + 1);
    pc->self_log = log(eps_s * pc->h);
    pc->L = 0;
    while ((8 << pc->L) < n) pc->L++;
    pc->gx = (double *)malloc(sizeof(double) * N);
    pc->gy = (double *)malloc(sizeof(double) * N);
    pc->rx = (double *)malloc(sizeof(double) * m);
    pc->ry = (double *)malloc(sizeof(double) * m);
    orc_grid_points(n, pc->gx, pc->gy);
    orc_ring_points(n, pc->rx, pc->ry);
    pc->tx = (double *)malloc(sizeof(double) * (N + m));
    pc->ty = (double *)malloc(sizeof(double) * (N + m));
    memcpy(pc->tx, pc->gx, sizeof(double) * N);
    memcpy(pc->ty, pc->gy, sizeof(double) * N);
    memcpy(pc->tx + N, pc->rx, sizeof(double) * m);
    memcpy(pc->ty + N, pc->ry, sizeof(double) * m);
    if (bem) {
        pc->LU = (double *)malloc(sizeof(double) * (size_t)m * m);
        pc->piv = (int *)malloc(sizeof(int) * m);
        orc_bem_matrix(n, pc->LU);
        if (orc_lu_factor(m, pc->LU, pc->piv) != 0) return NULL;
    }
    return pc;
}

void orc_pc_destroy(void *v)
{
    orc_pc *pc = (orc_pc *)v;
    if (!pc) return;
    free(pc->gx); free(pc->gy); free(pc->rx); free(pc->ry);
    free(pc->tx); free(pc->ty); free(pc->LU); free(pc->piv);
    free(pc);
}

/* volume potential of charges q at the given targets, by FMM or by direct sum */
static void pc_potential(const orc_pc *pc, int ns, const double *sx, const double *sy,
                         const double *q, int nt, const double *tx, const double *ty,
                         double *u)
{
    if (pc->exact)
        orc_direct(ns, sx, sy, q, nt, tx, ty, pc->self_log, u);
    else if (pc->theta > 0.0)
        orc_fmm_theta(pc->L, 0.5 * pc->h, 0.5 * pc->h, pc->n * pc->h, pc->p, pc->theta, ns, sx,
                      sy, q, nt, tx, ty, pc->self_log, u);
    else
        orc_fmm(pc->L, 0.5 * pc->h, 0.5 * pc->h, pc->n * pc->h, pc->p, ns, sx, sy, q,
                nt, tx, ty, pc->self_log, u);
}

/* z = P^{-1} r.  Optional outputs: phi_ring (4n), sigma (4n). */
int orc_pc_apply_ex(void *v, const double *r, double *z, double *phi_ring, double *sigma)
{
    orc_pc *pc = (orc_pc *)v;
    int n = pc->n, m = 4 * n;
    size_t N = (size_t)n * n;
    double h = pc->h;
    double *q = (double *)malloc(sizeof(double) * N);
    double *phi = (double *)malloc(sizeof(double) * (N + m));
    /* midpoint rule for the volume integral: q_j = h^2 r_j */
    for (size_t i = 0; i < N; ++i) q[i] = h * h * r[i];
    /* pass 1: volume potential at interior nodes and ring nodes */
    pc_potential(pc, (int)N, pc->gx, pc->gy, q, (int)(N + m), pc->tx, pc->ty, phi);
    memcpy(z, phi, sizeof(double) * N);
    if (phi_ring) memcpy(phi_ring, phi + N, sizeof(double) * m);
    if (pc->bem) {
        /* S sigma = -phi_ring */
        double *sg = (double *)malloc(sizeof(double) * m);
        for (int k = 0; k < m; ++k) sg[k] = -phi[N + k];
        orc_lu_solve(m, pc->LU, pc->piv, sg);
        if (sigma) memcpy(sigma, sg, sizeof(double) * m);
        /* pass 2: single layer with element weight h, evaluated at interior nodes */
        double *qs = (double *)malloc(sizeof(double) * m);
        for (int k = 0; k < m; ++k) qs[k] = h * sg[k];
        double *corr = (double *)malloc(sizeof(double) * N);
        pc_potential(pc, m, pc->rx, pc->ry, qs, (int)N, pc->gx, pc->gy, corr);
        for (size_t i = 0; i < N; ++i) z[i] += corr[i];
        free(sg); free(qs); free(corr);
    }
    free(q); free(phi);
    return 0;
}

int orc_pc_apply(void *v, const double *r, double *z)
{
    return orc_pc_apply_ex(v, r, z, NULL, NULL);
}

/* The boundary stage alone: sigma = -S^{-1} phi_ring (Sec. 4.3, the
 * collocation system with zero Dirichlet data), with the factors of S kept
 * by the preconditioner.  Returns -1 when it was built without bem. */
int orc_pc_bem_solve(void *v, const double *phi_ring, double *sigma)
{
    orc_pc *pc = (orc_pc *)v;
    if (!pc->bem) return -1;
    int m = 4 * pc->n;
    for (int k = 0; k < m; ++k) sigma[k] = -phi_ring[k];
    orc_lu_solve(m, pc->LU, pc->piv, sigma);
    return 0;
}

/* ======================================================================== */
/* Right-preconditioned FGMRES(m), modified Gram-Schmidt, Givens rotations.  */
/* pc == NULL means the identity preconditioner.  x holds x0 on entry.       */
/* Returns 0 when converged, 1 when maxit inner steps were spent.            */
/* ======================================================================== */
static double dotv(size_t N, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t i = 0; i < N; ++i) s += a[i] * b[i];
    return s;
}

int orc_fgmres(int n, void *pc, const double *b, double *x, double tol, int m,
               int maxit, int *iters_out, double *true_rel_out, double *hist)
{
    size_t N = (size_t)n * n;
    double *V = (double *)malloc(sizeof(double) * N * (m + 1));
    double *Z = (double *)malloc(sizeof(double) * N * m);
    double *w = (double *)malloc(sizeof(double) * N);
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1)), *yv = (double *)malloc(sizeof(double) * m);
    double bnorm = sqrt(dotv(N, b, b));
    int iters = 0, status = 1;
    if (bnorm == 0.0) { memset(x, 0, sizeof(double) * N); *iters_out = 0; *true_rel_out = 0.0; status = 0; goto done; }
    for (;;) {
        orc_stencil(n, x, w);
        for (size_t i = 0; i < N; ++i) w[i] = b[i] - w[i];
        double beta = sqrt(dotv(N, w, w));
        if (beta / bnorm <= tol) { status = 0; *true_rel_out = beta / bnorm; break; }
        if (iters >= maxit) { status = 1; *true_rel_out = beta / bnorm; break; }
        for (size_t i = 0; i < N; ++i) V[i] = w[i] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && iters < maxit; ++j) {
            double *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N;
            if (pc) orc_pc_apply(pc, vj, zj); else memcpy(zj, vj, sizeof(double) * N);
            orc_stencil(n, zj, w);
            for (int i = 0; i <= j; ++i) {
                double hij = dotv(N, w, V + (size_t)i * N);
                H[(size_t)i * m + j] = hij;
                for (size_t t = 0; t < N; ++t) w[t] -= hij * V[(size_t)i * N + t];
            }
            double hn = sqrt(dotv(N, w, w));
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn != 0.0)
                for (size_t t = 0; t < N; ++t) V[(size_t)(j + 1) * N + t] = w[t] / hn;
            /* apply the previous rotations, then build the new one */
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            double rr = sqrt(a * a + c * c);
            cs[j] = a / rr; sn[j] = c / rr;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters; k = j + 1;
            if (hist) hist[iters - 1] = fabs(g[j + 1]) / bnorm;
            if (fabs(g[j + 1]) / bnorm <= tol || hn == 0.0) break;
        }
        /* back substitution H y = g, then x += Z y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t < k; ++t) s -= H[(size_t)i * m + t] * yv[t];
            yv[i] = s / H[(size_t)i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (size_t t = 0; t < N; ++t) x[t] += yv[i] * Z[(size_t)i * N + t];
    }
    *iters_out = iters;
done:
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(yv);
    return status;
}

/* number of OpenMP threads a parallel region of the oracle uses */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
