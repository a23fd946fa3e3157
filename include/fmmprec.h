/*
 * fmmprec.h -- C ABI of the MI355X (gfx950) FMM-preconditioned Poisson solver.
 *
 * Method: Ibeid, Yokota, Pestana, Keyes, "Fast Multipole Preconditioners for
 * Sparse Matrices Arising from Elliptic Equations" (arXiv:1308.3339).
 *   - The linear system A x = b of Sec. 2.1 (eq. axb), here the 5-point
 *     finite-difference Laplacian on the unit square with Dirichlet data.
 *   - Only the action of the preconditioner P^{-1} is needed (Sec. 3.1), and
 *     it is applied from the right.
 *   - P^{-1} is the FMM-BEM preconditioner of Sec. 3.3 (Fig. 1): a volume
 *     potential u_i = sum_j f_j G_ij (Sec. 5.1, eq. volume_integral) evaluated
 *     by the FMM of Sec. 5, corrected by a boundary-element solve for zero
 *     Dirichlet data (Sec. 4.1, eqs. ubound and uinter).
 *   - Setup once, apply every iteration (Sec. 7.1: PCSetUp / PCApply).
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *     unless stated otherwise.  `stream` is a hipStream_t passed as void*
 *     (NULL = the default stream).
 *   - Grid arrays are row-major n x n: node (i, j), i, j = 0..n-1, lives at
 *     index j*n + i and at the point ((i+1)h, (j+1)h), h = 1/(n+1).
 *   - Ring arrays hold the 4n Dirichlet nodes next to the grid (corners
 *     excluded), counter-clockwise: bottom ((k+1)h, 0), right (1, (k+1)h),
 *     top ((n-k)h, 1), left (0, (n-k)h); node s*n + k for side s, k = 0..n-1.
 *   - nrhs > 1 means nrhs arrays stored back to back (stride n*n, or N).
 *   - Ownership: the caller owns all input/output buffers and keeps them
 *     alive until the stream work is done; the plan owns every workspace
 *     (expansions, tables, boundary inverse, Krylov basis) and
 *     fmm_destroy() frees it.
 *   - fmm_apply / fmm_precond_apply / fmm_stencil_apply are asynchronous and
 *     ordered on `stream`.  precond_gmres_solve synchronises `stream` before
 *     it returns (its result struct lives on the host).
 *   - A plan may be used by one stream at a time (calls that overlap on two
 *     streams race on the plan's workspace).
 *   - Errors are status codes; nothing is thrown across the ABI.  After a
 *     negative status the outputs are undefined and fmm_last_error() holds a
 *     message.
 */
#ifndef FMMPREC_H
#define FMMPREC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan fmm_plan; /* opaque, library-owned */

enum {
    FMM_OK = 0,
    FMM_NOT_CONVERGED = 1,  /* maxit spent; u holds the last iterate     */
    FMM_ERR_ARG = -1,       /* an argument failed validation            */
    FMM_ERR_DEVICE = -2,    /* a HIP call failed                        */
    FMM_ERR_ALLOC = -3,     /* device or host allocation failed         */
    FMM_ERR_NUMERIC = -4,   /* NaN/Inf met (right-hand side or Arnoldi) */
    FMM_ERR_UNSUPPORTED = -5 /* valid request this build does not serve  */
};

typedef enum { FMM_GRID = 0, FMM_POINTS = 1 } fmm_kind;

/* Arithmetic of the FMM.  FMM_FP64: everything in FP64.  FMM_FP32 (GRID
 * plans): the near field (P2P) and P2M run as FP32 matrix-core contractions
 * (each 64-term FP32 partial folded into FP64) and the multipole-to-local
 * translations in FP32 (the preconditioner's tunable accuracy, Sec. 6.2).
 * FMM_FP32 (POINTS plans): the near field runs pairwise in FP32 as in Secs.
 * 5.3 and 7.1 (FP32 offsets from the target leaf's centre, log2 from a
 * polynomial fit of log2(x)/(x - 1), Kahan-compensated sums; pairs whose
 * FP32 r^2 is below the smallest normal float are left out like the self
 * pair); P2M, M2M, M2L, L2L and L2P stay FP64.
 * FMM_SPLIT_FP16 (GRID plans): as FMM_FP32, but the near field, P2M and the
 * multipole-to-local translations take each operand as an FP16 pair
 * x = hi + lo (charges and multipoles scaled per tile by a power of two, the
 * translation operators split at setup) and sum hi*hi + hi*lo + lo*hi on the
 * FP16 matrix cores with FP32 accumulation (about 2^-22 relative per
 * product).
 * FMM_SPLIT_BF16 (GRID plans): the same with BF16 pairs on the BF16 matrix
 * cores, summing all four products hi*hi + hi*lo + lo*hi + lo*lo (about
 * 2^-16 relative per product, the pairs' representation error).
 * In every precision M2M, L2L, L2P, the boundary correction, the stencil and
 * Krylov stay FP64, and the flexible outer iteration reaches the same FP64
 * residual. */
typedef enum {
    FMM_FP64 = 0,
    FMM_FP32 = 1,
    FMM_SPLIT_BF16 = 2,
    FMM_SPLIT_FP16 = 3
} fmm_precision;

/* The problem the plan is built for.
 *   GRID:   n = interior points per side, n = 8 * 2^L with 0 <= L <= 12 (n <= 32768,
 *           so that n^2 < 2^32); x, y unused.
 *           The quadtree root is the square [h/2, 1-h/2]^2, whose leaves are
 *           the 8 x 8 blocks of the grid.
 *   POINTS: n = number of points N >= 1; x, y = DEVICE arrays of N
 *           coordinates inside the root square [x0, x0+side] x [y0, y0+side]
 *           (side > 0).  They are read during fmm_setup only.  The tree has
 *           L = ceil(log4(N/64)) levels (at least 0); a point belongs to leaf
 *           min(max(floor((x - x0)/side * 2^L), 0), 2^L - 1) per axis. */
typedef struct {
    int32_t kind;   /* fmm_kind */
    int64_t n;
    const double *x;
    const double *y;
    double x0, y0, side;
} fmm_problem;

/* FMM parameters.
 *   p        number of expansion coefficients, M_0..M_{p-1} (Sec. 5.3), 2..20.
 *            Above 20 the downward pass's LDS (16 (4p^2 + 216p) bytes per
 *            block, 176 KiB at p = 32) and M2L's source tile (16 p (16 + 4K)^2
 *            bytes, above 160 KiB for p > 25 with the list rule) outgrow a
 *            compute unit's 160 KiB; p = 20 already puts the list rule's
 *            truncation error near 1e-11, three digits above FP64 rounding.
 *   leaf     points per leaf side squared; must be 64 (8 x 8 grid blocks).
 *   prec     fmm_precision (FMM_FP32 for GRID and POINTS plans, FMM_SPLIT_BF16
 *            and FMM_SPLIT_FP16 for GRID plans).
 *   bem      GRID: 1 = boundary correction on (Sec. 4), 0 = free-space
 *            volume potential only.  Ignored for POINTS.
 *   self_eps GRID: the singular self term is G_self = -(1/2pi) log(self_eps h)
 *            (Sec. 4.2 smoothing read as a self-cell value); 0 selects the
 *            default exp(-gamma)/(2 sqrt 2) = 0.1985..., which matches the
 *            5-point lattice Green's function at short range.
 *   theta    well-separatedness.  0: the interaction lists of Sec. 5.2 (the
 *            children of the parent's 3x3 neighbourhood that are not
 *            adjacent; near field = 3x3 leaves).  In [0.3, 1]: the multipole
 *            acceptance criterion of the dual tree traversal (Sec. 5.2): two
 *            cells of one level interact by M2L when the sum of their radii
 *            (half diagonals) is below theta times their centre distance,
 *            failing pairs are split together, failing leaf pairs are P2P.
 *            On the uniform tree the near field is then the disk of leaves
 *            |d|^2 <= 2/theta^2 and the lists the parent disk's children
 *            outside it; theta > 1/sqrt(2) gives the list rule again.
 *            Smaller theta trades more near-field and M2L work for accuracy
 *            at a given p (p = 6, theta = 0.4 gives about six digits).
 *            theta < 1/sqrt(2) requires FMM_FP64 (any kind) or FMM_FP32 (GRID:
 *            the disk's near field on the FP32 matrix cores, M2L in FP32),
 *            p <= 12 and p (16 + 4K)^2 * 16 <= 160 KiB, K = floor(sqrt(2)/theta)
 *            (so p <= 10 for theta < 0.354); otherwise FMM_ERR_UNSUPPORTED. */
typedef struct {
    int32_t p;
    int32_t leaf;
    int32_t prec;
    int32_t bem;
    double self_eps;
    double theta;
} fmm_params;

/* Krylov parameters: tol > 0 (relative true residual ||b - Ax||/||b||),
 * restart in [1, 32], maxit >= 1 (total inner iterations).  The restart
 * length is capped at 32 by the Arnoldi sweeps: each step orthogonalises in
 * one pass over the basis that keeps 2j + 3 FP64 partial sums and j basis
 * values per lane in registers (about 210 VGPRs at j = 31), and the group
 * solver keeps each instance's rotated Hessenberg columns, (m + 1) x m
 * doubles, in one device record.  The FMM-preconditioned iteration counts
 * of Sec. 6 are 5-7 at every mesh size (Tables 1, 3 and 4; 7-8 here to
 * 1e-8 up to 2048^2), far inside one cycle of 32; FMM_ERR_ARG otherwise. */
typedef struct {
    double tol;
    int32_t restart;
    int32_t maxit;
} gmres_params;

/* HOST struct filled by precond_gmres_solve. */
typedef struct {
    int32_t iters;        /* inner iterations (= preconditioner applications) */
    int32_t restarts;     /* completed restart cycles                         */
    double est_rel_res;   /* Givens estimate at the last inner iteration      */
    double true_rel_res;  /* ||b - A x|| / ||b|| recomputed at exit           */
} gmres_result;

/* Builds a plan (PCSetUp, Sec. 7.1): tree, operator tables, workspace and,
 * for GRID with bem=1, the inverse of the boundary collocation matrix.
 * `problem` and `params` are HOST pointers.  Synchronises `stream`.
 * Returns FMM_OK and *out, or an error with *out = NULL. */
int fmm_setup(const fmm_problem *problem, const fmm_params *params, void *stream,
              fmm_plan **out);

/* Volume potential by FMM (Sec. 5.1 eq. volume_integral, Sec. 5.3):
 *   GRID:   u_i = sum_j q_j G(x_i - x_j) over the n*n nodes with
 *           G = -(1/2pi) log r and the self term q_i G_self.
 *   POINTS: u_i = sum_{j != i} q_j G(x_i - x_j) in the caller's point order.
 * q and u hold nrhs arrays of n*n (GRID) or N (POINTS) doubles; u must not
 * alias q. */
int fmm_apply(fmm_plan *plan, const double *q, double *u, int nrhs, void *stream);

/* The tree order of a POINTS plan (Sec. 5.1, built on the device by
 * fmm_setup): points sorted by leaf, leaves in Morton order (bit b of the
 * leaf column at bit 2b, bit b of the leaf row at bit 2b + 1), points of
 * one leaf in their original order.  perm: N int32 (DEVICE), perm[i] = the
 * caller's index of the point at sorted position i; leaf_start: 4^L + 1
 * int32 (DEVICE), leaf_start[m] = first sorted position of the leaf with
 * Morton index m, leaf_start[4^L] = N, L = ceil(log4(N/64)) (at least 0).
 * Either pointer may be NULL (not both).  Asynchronous on `stream`. */
int fmm_points_order(fmm_plan *plan, int32_t *perm, int32_t *leaf_start, void *stream);

/* z = P^{-1} r (PCApply, Sec. 3.3 Fig. 1), GRID plans only:
 *   q = h^2 r (midpoint rule for the volume integral of Sec. 4.1),
 *   phi = FMM volume potential of q at the interior and ring nodes,
 *   bem=1: sigma = -S^{-1} phi_ring (collocation, Sec. 4.3) and
 *          z = phi + sum_l h sigma_l G(x - y_l) by a second FMM pass;
 *   bem=0: z = phi.
 * r and z hold nrhs grids; z must not alias r. */
int fmm_precond_apply(fmm_plan *plan, const double *r, double *z, int nrhs, void *stream);

/* As fmm_precond_apply for one right-hand side, also returning the ring
 * potential phi_ring (4n) and the boundary density sigma (4n) in ring order
 * (sigma is left untouched when bem=0).  Either extra pointer may be NULL. */
int fmm_precond_stages(fmm_plan *plan, const double *r, double *z, double *phi_ring,
                       double *sigma, void *stream);

/* w = A v, the 5-point Laplacian with zero Dirichlet data (Sec. 2.1):
 * (Av)_ij = (4 v_ij - v_{i-1,j} - v_{i+1,j} - v_{i,j-1} - v_{i,j+1}) / h^2.
 * GRID plans only; nrhs grids; w must not alias v. */
int fmm_stencil_apply(fmm_plan *plan, const double *v, double *w, int nrhs, void *stream);

/* Solves A u = b (Sec. 2.1, eq. axb) with right-preconditioned
 * FGMRES(restart) -- Sec. 3.1: the preconditioner only enters through its
 * action, which may change from one iteration to the next -- and P^{-1} of
 * fmm_precond_apply (GRID plans only):
 *   b = f + (boundary values g at the neighbouring ring nodes) / h^2,
 *   f: n*n grid (device); g: 4n ring values (device) or NULL for zero data;
 *   u: on entry the initial guess x0, on exit the solution;
 *   stop when ||b - A u|| / ||b|| <= tol (Givens estimate, then confirmed
 *   with an explicit residual; restart from the current u otherwise).
 * Returns FMM_OK, FMM_NOT_CONVERGED (maxit spent; u = last iterate and *res
 * valid) or an error.  `prm` and `res` are HOST pointers; prm may be NULL
 * (tol 1e-8, restart 30, maxit 600); res may be NULL. */
int precond_gmres_solve(fmm_plan *plan, const double *f, const double *g, double *u,
                        const gmres_params *prm, gmres_result *res, void *stream);

/* Many independent solves at once (GRID plans, sizes may differ): instance
 * i solves A u[i] = f[i] on plans[i] (zero ring data) with the settings of
 * precond_gmres_solve.  plans, f, u, res and elapsed_ms are HOST arrays of
 * count entries (f[i], u[i] device arrays as for precond_gmres_solve; res
 * and elapsed_ms may be NULL); the plans must be distinct.  Instances whose
 * plans describe the same problem (n, p, prec, theta, self_eps, bem) are
 * solved as groups of up to 16: every launch of an Arnoldi step (the whole
 * preconditioner, both orthogonalisation sweeps) covers the group, and the
 * Givens rotations and convergence tests run on the device, so a finished
 * instance turns the group's later launches into no-ops for itself.  A group
 * runs on the plan of its first instance (whose workspace then holds the
 * group's Krylov bases) and on that plan's stream, after the work already on
 * `stream`; a host loop advances whichever group's last step has completed,
 * so groups of different sizes overlap on the GPU.  elapsed_ms[i] = host
 * time from the call to the end of the cycle in which instance i converged.
 * flags: FMM_BATCH_GRAPHS replays each step (and each cycle's end) of a
 * group from a HIP graph captured the first time it runs;
 * FMM_BATCH_SEPARATE runs one solve per plan instead (each on its own
 * stream, Givens rotations on the host), the layout before groups.
 * `stream` waits for every instance before later work.  Returns FMM_OK when
 * every instance converged, FMM_NOT_CONVERGED when one did not, or an
 * error. */
enum { FMM_BATCH_GRAPHS = 1, FMM_BATCH_SEPARATE = 2 };
int precond_gmres_solve_batch(fmm_plan *const *plans, int32_t count, const double *const *f,
                              double *const *u, const gmres_params *prm, gmres_result *res,
                              double *elapsed_ms, int32_t flags, void *stream);

/* nrhs right-hand sides on one plan at once (GRID plans; the many
 * right-hand sides of Sec. 3.1's solve): f and u hold nrhs grids of n*n
 * doubles back to back (u: initial guesses on entry, solutions on exit),
 * res (HOST, may be NULL) nrhs results.  Solved in groups of up to 16 as in
 * precond_gmres_solve_batch (one launch per stage for the group, Givens
 * rotations and convergence tests on the device); flags: FMM_BATCH_GRAPHS.
 * Synchronises `stream`.  Arguments and return codes otherwise as for
 * precond_gmres_solve. */
int precond_gmres_solve_multi(fmm_plan *plan, int32_t nrhs, const double *f, double *u,
                              const gmres_params *prm, gmres_result *res, int32_t flags,
                              void *stream);

/* Autotuner: times the Krylov sweeps of this plan's grid with candidate
 * block counts (64 .. 4096; the fastest of three calls each, in three rounds
 * over the candidates) and keeps the fastest for later solves; the choice is
 * returned in *vec_blocks (HOST, may be NULL).  Synchronises `stream`.  GRID
 * plans only. */
int fmm_tune(fmm_plan *plan, void *stream, int32_t *vec_blocks);

/* M2L tile shape (Sec. 5.3 item 3, the translations of every level in one
 * launch).  The launch has one block per 16 x 16 tile of target cells and
 * list share: with split S each tile's interaction lists are cut into S
 * shares of consecutive entries, S blocks translate one share each into
 * their own part of the M2L sums, and the downward pass adds the S parts in
 * order (so results are deterministic; they change with S only by the order
 * of the additions).  S in {1, 2, 4, 8}; the plan starts with the smallest S
 * that gives every second compute unit a block (2 S tiles >= compute units:
 * the 2048^2 tree's 343 tiles take S = 1, the 1024^2 tree's 87 take S = 2).
 * A call over nrhs stacked right-hand sides (or a group of a batch) takes
 * S / nrhs (rounded down to a power of two, at least 1), since the
 * right-hand sides already multiply the blocks; its results then agree with
 * single calls to rounding rather than bit for bit.
 *   fmm_tune_m2l: times the M2L and downward launches of the plan for each S
 *     on `stream` (the fastest of three calls, in three rounds over the four
 *     values), keeps the fastest S, writes it to *split (HOST, may be NULL);
 *     synchronises `stream`.
 *   fmm_set_m2l_split: sets S (FMM_ERR_ARG otherwise); synchronises the
 *     device (the buffer of M2L sums may grow).
 *   fmm_get_m2l_split: the plan's current S into *split (HOST).
 * Captured solver graphs of the plan are dropped by the first two. */
int fmm_tune_m2l(fmm_plan *plan, void *stream, int32_t *split);
int fmm_set_m2l_split(fmm_plan *plan, int32_t split);
int fmm_get_m2l_split(const fmm_plan *plan, int32_t *split);

/* Variable-coefficient operator of Sec. 6.4, -div(a grad u), in flux form
 * on the plan's grid (GRID plans only), zero Dirichlet data:
 *   h^2 (A v)_ij = ax[j][i+1] (v_ij - v_{i+1,j}) + ax[j][i] (v_ij - v_{i-1,j})
 *                + ay[j+1][i] (v_ij - v_{i,j+1}) + ay[j][i] (v_ij - v_{i,j-1}),
 * v = 0 outside the grid.  ax: n x (n+1) face values, row-major, ax[j][i] =
 * a((i + 1/2) h, (j + 1) h) between nodes i-1 and i of row j; ay: (n+1) x n,
 * ay[j][i] = a((i + 1) h, (j + 1/2) h) between rows j-1 and j.  Device
 * arrays, caller-owned; a > 0 is the caller's to ensure. */
int fmm_stencil_var_apply(fmm_plan *plan, const double *ax, const double *ay, const double *v,
                          double *w, void *stream);

/* Solves A u = f for the variable-coefficient A above (zero Dirichlet
 * data) with right-preconditioned FGMRES(restart), preconditioned by the
 * plan's constant-coefficient FMM-BEM operator: for smooth a the two are
 * spectrally equivalent (Sec. 6.4).  Arguments, stopping rule and return
 * codes as for precond_gmres_solve. */
int precond_gmres_solve_var(fmm_plan *plan, const double *ax, const double *ay, const double *f,
                            double *u, const gmres_params *prm, gmres_result *res, void *stream);

/* Adjoint solve for gradients through precond_gmres_solve: lambda solves
 * A^T lambda = g (GRID plans only).  A is the symmetric 5-point matrix of
 * Sec. 2.1, and b depends on f through the identity, so for a loss L(u)
 * with u = A^{-1} b(f): dL/df = lambda with g = dL/du.  The call runs the
 * same right-preconditioned FGMRES as precond_gmres_solve on the right-hand
 * side g (zero ring data); lambda is the initial guess on entry and the
 * result on exit.  prm, res: as for precond_gmres_solve. */
int precond_gmres_solve_adjoint(fmm_plan *plan, const double *g, double *lambda,
                                const gmres_params *prm, gmres_result *res, void *stream);

/* Gaussian-bump source on the plan's grid (GRID plans only; the source model
 * of the differentiation workload, not part of the paper):
 *   f_i = sum_{k < K} a_k exp(-|x_i - c_k|^2 / (2 w_k^2)),
 * x_i the interior nodes ((i+1)h, (j+1)h).  cx, cy, w, a: K device doubles
 * (1 <= K <= 256, w_k > 0 is the caller's to ensure); f: n*n device doubles. */
int fmm_bumps_eval(fmm_plan *plan, int32_t K, const double *cx, const double *cy,
                   const double *w, const double *a, double *f, void *stream);

/* Gradients of sum_i g_i f_i (f as in fmm_bumps_eval) with respect to the
 * bump parameters, given g = dL/df (n*n device doubles):
 *   gcx_k = a_k / w_k^2 sum_i g_i e_ik (x_i - cx_k), gcy_k likewise,
 *   gw_k  = a_k / w_k^3 sum_i g_i e_ik |x_i - c_k|^2,  ga_k = sum_i g_i e_ik,
 * e_ik = exp(-|x_i - c_k|^2 / (2 w_k^2)).  Outputs: K device doubles each
 * (any of them may be NULL).  Sums run in a fixed order (bitwise
 * reproducible).  The plan keeps a small reduction workspace. */
int fmm_bumps_grad(fmm_plan *plan, int32_t K, const double *cx, const double *cy,
                   const double *w, const double *a, const double *g, double *gcx,
                   double *gcy, double *gw, double *ga, void *stream);

/* As fmm_bumps_grad, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the call allocates nothing.  Its partial sums live in a static workspace
 * of the library, 1 MiB per device (the partials of K <= 256 bumps), which
 * each device the library runs on keeps until the process ends; larger K
 * is rejected with FMM_ERR_ARG.  Every call on one device shares that
 * workspace and fully overwrites the part it reads, so nothing carries over
 * between calls, but calls that overlap on one device (two streams, or two
 * threads) race and must be ordered by the caller.  Arguments, outputs and
 * results are those of fmm_bumps_grad (bitwise: the same kernels). */
int fmm_bumps_grad_noalloc(fmm_plan *plan, int32_t K, const double *cx, const double *cy,
                           const double *w, const double *a, const double *g, double *gcx,
                           double *gcy, double *gw, double *ga, void *stream);

/* Per-stage device timing (tracing support).  Stages of an apply or solve:
 * P2M (a pass of its own in FMM_FP32 plans), M2M, M2L, L2L (Sec. 5.3 items
 * 1-4; L2L also covers the far-field L2P sweep when no boundary pass
 * follows), LEAF (P2P near field of Sec. 5.1 and, in FMM_FP64 plans, the
 * P2M of item 1), RING (potential at the ring nodes), BEM (boundary solve,
 * Sec. 4.3), PASS2 (boundary-source FMM pass and the far-field L2P sweep of
 * both passes), STENCIL (A v and residuals), ARNOLDI (orthogonalisation and
 * updates). */
enum {
    FMM_STAGE_P2M = 0, FMM_STAGE_M2M, FMM_STAGE_M2L, FMM_STAGE_L2L, FMM_STAGE_LEAF,
    FMM_STAGE_RING, FMM_STAGE_BEM, FMM_STAGE_PASS2, FMM_STAGE_STENCIL, FMM_STAGE_ARNOLDI,
    FMM_STAGE_COUNT
};

/* HOST struct: accumulated GPU milliseconds and launch counts per stage. */
typedef struct {
    double ms[16];
    int64_t launches[16];
} fmm_profile_stats;

/* Enables hipEvent timing of the stages in stage_mask (bit s = stage s;
 * 0 disables) and clears the accumulated statistics.  Events are recorded
 * on the stream of each later call, around that stage's launches only, so
 * an enabled stage adds two event records per occurrence. */
int fmm_profile(fmm_plan *plan, uint32_t stage_mask);

/* Waits for the recorded events and returns the accumulated statistics
 * (HOST pointer). */
int fmm_profile_read(fmm_plan *plan, fmm_profile_stats *out);

/* Frees the plan and everything it owns.  NULL is accepted. */
int fmm_destroy(fmm_plan *plan);

/* Message for the last error on this plan (or of the last failed fmm_setup
 * when plan is NULL).  The string is owned by the library. */
const char *fmm_last_error(const fmm_plan *plan);

/* Library version string, e.g. "fmmprec 0.1 gfx950". */
const char *fmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMMPREC_H */
