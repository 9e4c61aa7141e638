/*
 * mfr.h -- matrix-free NGF + curvature image registration on MI355X (gfx950).
 *
 * C ABI of the library libmfr.so.  It evaluates the discretised objective
 * J(y) = D(y) + alpha S(y) of Sec. 2.2 (eq. discreteenergy: the normalized
 * gradient fields distance D of eq. NGF_discretized and the curvature
 * regulariser S of eq. CURV_discretized), its gradient and the Gauss-Newton
 * Hessian-vector product of Sec. 3-4 (eq. NGF_discretized_gradient,
 * eq. NGF_discretized_hessian, eq. curvatureMF, eq. curv_hessMult), and runs
 * the Gauss-Newton / conjugate-gradient loop of Sec. 2.3 on a coarse-to-fine
 * pyramid.  Every arithmetic step runs in hand-written HIP kernels.
 *
 * Conventions (all calls):
 *  - Images are contiguous float32 arrays [m_z][m_y][m_x] (x fastest): the
 *    lexicographic order of Sec. 2.2.  Voxel (a,b,c) has centre
 *    ((a+1/2)h_x, (b+1/2)h_y, (c+1/2)h_z).
 *  - Node vectors (displacement u, directions p, results) are contiguous
 *    float32 arrays [3][n_z][n_y][n_x]: all x components, then y, then z
 *    (the component-major order of Sec. 2.2).  Node (i,j,k) sits at
 *    (i hy_x, j hy_y, k hy_z) with hy = m h / (n - 1): the nodal grid spans
 *    the image domain.
 *  - The unknown is the DISPLACEMENT u = y - x^y (Sec. 2.2); derivatives with
 *    respect to u and y coincide.
 *  - Two-dimensional problems (the d = 2 case of Sec. 2.2; the paper's GPU
 *    experiments of Sec. 6.3 are 2D) have one image cell and one node along z:
 *    m[2] = my[2] = 1 (mT[2] 0 or 1; h[2], hT[2] are ignored).  Images are
 *    [m_y][m_x], node vectors [2][n_y][n_x] (x components, then y), the
 *    interpolation is bilinear, four short differences per pixel, the 5-point
 *    Laplacian, hbar = h_x h_y.  They take the NGF distance and the curvature
 *    regulariser; every single-pair call accepts them except the
 *    learned-preconditioner calls (MFR_EINVAL), and the batched path takes
 *    three-dimensional problems only.
 *  - Every pointer argument named R, T, u, p, q, g, b, s, diag or workspace is
 *    a DEVICE pointer (hipMalloc / torch CUDA memory), 4-byte aligned (the
 *    workspace 256-byte aligned), owned by the caller and only borrowed for the
 *    duration of the call -- except R and T, borrowed until the next
 *    mfr_set_images or mfr_destroy.  Pointers to mfr_* structs and to double
 *    results are HOST pointers.  The library never allocates device memory.
 *  - Work is enqueued on the HIP stream given to mfr_create.  Calls that return
 *    host scalars (J, D, S, PCG info) synchronise that stream; the others
 *    return once their kernels are enqueued.
 *  - A context is not thread-safe; separate contexts on separate streams are.
 *  - Every call validates its arguments before any launch and returns an
 *    mfr_status; mfr_last_error() gives a thread-local message for the last
 *    non-OK status.  No C++ exception crosses the ABI.
 */
#ifndef MFR_H
#define MFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFR_ABI_VERSION 4

/* Regularisers (mfr_grid.regulariser). */
#define MFR_REG_CURVATURE 0   /* curvature, eq. CURV_discretized (the paper's)                  */
#define MFR_REG_DIFFUSIVE 1   /* diffusive hbar^y/2 sum_d sum_edges ((u_m - u_n)/hy_k)^2 over
                                 neighbouring nodes (Sec. 4.4); Hessian -hbar^y L               */
#define MFR_REG_ELASTIC 2     /* linear elastic (Sec. 4.4): lame_mu times the diffusive term plus
                                 hbar^y/2 (lame_lambda + lame_mu) sum_cells (div u)^2, the
                                 divergence per cell of the nodal grid being sum_d of the mean
                                 of its four edge differences along d over hy_d                 */

/* Distance measures (mfr_grid.distance). */
#define MFR_DIST_NGF 0   /* normalized gradient fields, eq. NGF_discretized (the paper's) */
#define MFR_DIST_SSD 1   /* sum of squared differences hbar/2 sum_i (T(P y)_i - R_i)^2
                            (Sec. 4.4: the residual Jacobian dr/dT is the identity)    */

typedef enum {
  MFR_OK = 0,
  MFR_EINVAL = -1,        /* invalid argument (sizes, parameters, null or misaligned pointer) */
  MFR_ENOMEM = -2,        /* workspace smaller than the size query returned                   */
  MFR_EHIP = -3,          /* a HIP runtime call or kernel launch failed                       */
  MFR_ENONFINITE = -4,    /* a scalar result (J, D, S, dot product) is NaN or infinite       */
  MFR_ELINESEARCH = -5,   /* Armijo line search found no sufficient decrease                  */
  MFR_EBREAKDOWN = -6,    /* reserved: CG breakdown is reported in mfr_pcg_info.flag          */
  MFR_ENOTCONV = -7       /* a CG solve reached max_iter above rtol and the caller asked for
                             convergence (mfr_pcg_opts.require_converged); info is filled and
                             s holds the last iterate                                         */
} mfr_status;

/* Problem description (Sec. 2.2; notation table).  Sizes and spacings are
 * given per dimension in the order x, y, z. */
typedef struct {
  int32_t m[3];     /* image grid cells; 2 <= m (m[2] = my[2] = 1: a 2D problem)              */
  double h[3];      /* image grid spacing; > 0                                                */
  int32_t my[3];    /* deformation grid NODES; 2 <= my and my - 1 <= m (Sec. 2.2)             */
  int32_t mT[3];    /* template grid cells (all 0: same as m)                                 */
  double hT[3];     /* template grid spacing (all 0: same as h)                               */
  double tau;       /* NGF edge parameter of the template, > 0 (eq. ngf; ignored for SSD)    */
  double rho;       /* NGF edge parameter of the reference, > 0 (eq. ngf; ignored for SSD)   */
  double alpha;     /* curvature weight, >= 0 (eq. optimizationProblem)                       */
  int32_t distance; /* MFR_DIST_NGF (0) or MFR_DIST_SSD (1)                                   */
  int32_t regulariser; /* MFR_REG_CURVATURE (0), MFR_REG_DIFFUSIVE (1) or MFR_REG_ELASTIC (2)  */
  double lame_mu;      /* elastic only: > 0                                                  */
  double lame_lambda;  /* elastic only: lame_lambda + lame_mu >= 0                           */
} mfr_grid;

typedef struct mfr_ctx mfr_ctx;   /* opaque host-side context; owns no device memory */

int mfr_abi_version(void);
const char* mfr_last_error(void);

/* Bytes of device workspace a context for `grid` needs (tile partial sums,
 * reduction partials, lookup tables, the template copy with a zero border
 * that realises its Dirichlet extension, and the six node vectors of PCG). */
mfr_status mfr_workspace_size(const mfr_grid* grid, size_t* bytes);

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = default
 * stream) and to a caller-owned device workspace of at least
 * mfr_workspace_size bytes.  *out receives the context. */
mfr_status mfr_create(const mfr_grid* grid, void* hip_stream, void* workspace, size_t ws_bytes,
                      mfr_ctx** out);
void mfr_destroy(mfr_ctx* ctx);

/* Bind the reference R [m_z][m_y][m_x] and template T [mT_z][mT_y][mT_x]
 * (device, float32).  Copies T into the workspace with a two-cell zero border
 * (the template's zero Dirichlet extension, Sec. 2.2). */
mfr_status mfr_set_images(mfr_ctx* ctx, const float* R, const float* T);

/* J = D + alpha S at displacement u (eq. discreteenergy).  D follows
 * eq. NGF_discretized_ri (SSD: hbar/2 sum_i r_i^2 with r = T(P y) - R),
 * S eq. CURV_discretized (diffusive: see MFR_REG_DIFFUSIVE).  Any of J, D, S may be NULL.  Sums are accumulated
 * in float64.  Synchronises the stream. */
mfr_status mfr_objective(mfr_ctx* ctx, const float* u, double* J, double* D, double* S);

/* g = grad D + alpha grad S at u (eq. gradNGF with the transposed grid
 * conversion of Sec. 4.3, and eq. curvatureMF; SSD: hbar P^T (g_T r) with
 * g_T the template derivative, Sec. 4.4).  g: device [3][n].  If J (host) is
 * not NULL it receives J(u) (and the stream is synchronised).  The argument
 * order (u, J, g) is that of mfr_objective's results followed by the vector. */
mfr_status mfr_gradient(mfr_ctx* ctx, const float* u, double* J, float* g);

/* q = (H + alpha nabla^2 S) p with H the Gauss-Newton matrix of D at u
 * (eq. NGF_discretized_hessian, evaluated matrix-free as in eq. hessMult /
 * eq. drTdr; SSD: hbar P^T dT^T dT P, Sec. 4.4) and
 * nabla^2 S = 2 hbar^y L^T L (eq. curv_hessMult).
 * q must not alias u or p.  Asynchronous. */
mfr_status mfr_hess_vec(mfr_ctx* ctx, const float* u, const float* p, float* q);

/* Twins of mfr_objective and mfr_gradient for HIP graph capture (eq.
 * discreteenergy, eq. gradNGF, as above): the same kernels, with the scalars
 * written by the device into caller memory instead of returned, so nothing
 * synchronises or reads back and the calls can be captured together with
 * mfr_hess_vec and mfr_jacobi_diag.  out: device double[3] = {J, D, S}; J of
 * mfr_gradient_async: device double[1] or NULL.  Values equal those of the
 * synchronous calls bit for bit.  A non-finite J is written as it is (the
 * synchronous calls return MFR_ENONFINITE for it).  A captured graph uses the
 * context's workspace: replay it on the context's stream (or ordered with
 * it), never while other calls on the context run.  Asynchronous. */
mfr_status mfr_objective_async(mfr_ctx* ctx, const float* u, double* out);
mfr_status mfr_gradient_async(mfr_ctx* ctx, const float* u, double* J, float* g);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * q of mfr_hess_vec for `grid`, images R, T, displacement u and direction p,
 * with the workspace taken from a fixed device array of
 * MFR_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends.  Same kernels, same result bit for bit as
 * mfr_create + mfr_set_images + mfr_hess_vec with the same tile configuration.
 * Allocates no device memory and needs no context or workspace.  All pointers
 * are device pointers on the current device; work is enqueued on hip_stream,
 * which must belong to that device.  Returns MFR_ENOMEM if the problem's
 * workspace (mfr_workspace_size) exceeds the array.  Every call on one GPU
 * uses the same array: calls that overlap in time (other streams, other host
 * threads) race and must not be issued; calls in order on one stream are
 * safe, each one rewriting what it reads.  Asynchronous after the table
 * uploads of its set-up, which synchronise the stream. */
#define MFR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mfr_status mfr_hess_vec_noalloc(const mfr_grid* grid, void* hip_stream, const float* R, const float* T,
                                const float* u, const float* p, float* q);

/* diag = diag(H + alpha nabla^2 S) at u, exactly (the Jacobi preconditioner
 * of the conjugate-gradient solve; the paper leaves CG unpreconditioned).
 * Entries may be 0 when alpha = 0.  Asynchronous. */
mfr_status mfr_jacobi_diag(mfr_ctx* ctx, const float* u, float* diag);

typedef struct {
  int32_t max_iter;   /* >= 0                                                   */
  double rtol;        /* stop when ||b - A s_k|| / ||b|| <= rtol (recursive residual) */
  int32_t precond;    /* 0 none (plain CG), 1 Jacobi, 2 learned (flexible CG; needs a
                         preconditioner attached with mfr_attach_pc)            */
  int32_t fallback_iters; /* precond 2 only: after this many iterations without
                         convergence, continue with Jacobi-PCG from the current
                         iterate (0: never)                                      */
  int32_t require_converged; /* != 0: return MFR_ENOTCONV when max_iter is reached
                         with the relative residual above rtol (flag 1)          */
} mfr_pcg_opts;

typedef struct {
  int32_t iters;      /* iterations performed                                    */
  double relres;      /* final relative residual                                 */
  int32_t flag;       /* 0 converged, 1 max_iter reached, 2 breakdown (p^T A p <= 0 or not finite) */
  int32_t used_fallback; /* 1 if a learned solve switched to Jacobi              */
} mfr_pcg_info;

/* Solve (H + alpha nabla^2 S) s = b at u by preconditioned CG from s = 0
 * (Sec. 2.3.1: the Newton equation solved with CG).  Vectors in float32, dot
 * products and step lengths in float64.  s: device [3][n].  With precond 2 the
 * direction update is the flexible (Polak-Ribiere) one, since the learned
 * preconditioner is nonlinear.  The Jacobi preconditioner is the exact
 * diagonal with zero entries (possible only for alpha = 0) taken as 1.  The
 * convergence test runs on the device; the call synchronises once per eight
 * iterations and at the end.  On a breakdown (flag 2) the iterate is the one
 * before the failing step. */
mfr_status mfr_pcg_solve(mfr_ctx* ctx, const float* u, const float* b, float* s,
                         const mfr_pcg_opts* opts, mfr_pcg_info* info);

/* Twin of mfr_pcg_solve for HIP graph capture (Sec. 2.3.1, as above), precond 0
 * or 1: it enqueues the whole sequence of max_iter iterations with no host
 * read; the convergence test runs on the device and the iterations after it
 * has stopped the solve do nothing, so s equals that of mfr_pcg_solve bit for
 * bit.  info: device double[3] = {iterations, relative residual, flag (0, 1,
 * 2 as in mfr_pcg_info)}.  A right-hand side that is not finite shows as a
 * non-finite relative residual (the synchronous call returns MFR_ENONFINITE);
 * require_converged is refused.  Every launch of the sequence costs its launch
 * latency even after convergence: max_iter bounds the work.  A captured graph
 * uses the context's workspace (replay it on the context's stream).
 * Asynchronous. */
mfr_status mfr_pcg_solve_async(mfr_ctx* ctx, const float* u, const float* b, float* s, const mfr_pcg_opts* opts,
                               double* info);

typedef struct {
  int32_t pcg_max;     /* CG iterations                                              */
  double pcg_rtol;     /* CG relative residual tolerance (0: always pcg_max steps)   */
  int32_t precond;     /* 0 none, 1 Jacobi, 2 learned (attached preconditioner)      */
  double armijo_c1;    /* sufficient-decrease constant in [0, 1) (e.g. 1e-4)         */
  int32_t armijo_max;  /* trial step lengths 1, 1/2, 1/4, ... before giving up, >= 1 */
  int32_t fallback_iters; /* as in mfr_pcg_opts                                      */
} mfr_gn_opts;

typedef struct {
  double J_before;     /* J(u) on entry                                              */
  double J_after;      /* J at the accepted point (= J_before if none accepted)      */
  double eta;          /* accepted step length (0 if the line search failed)         */
  double slope;        /* grad J . s                                                 */
  int32_t pcg_iters;
  double pcg_relres;
  int32_t pcg_flag;
  int32_t accepted;    /* 1 if u was updated                                         */
  int32_t ls_trials;   /* objective evaluations spent in the line search             */
} mfr_gn_info;

/* One Gauss-Newton step at u (Sec. 2.3.1): gradient, (H + alpha nabla^2 S) s =
 * -grad J by (P)CG, Armijo line search eta = 1, 1/2, ... on J(u + eta s), and
 * u <- u + eta s if a step is accepted.  u: device [3][n], updated in place.
 * A failed line search is not an error: info->accepted = 0 and u is unchanged.
 * Synchronises the stream. */
mfr_status mfr_gn_step(mfr_ctx* ctx, float* u, const mfr_gn_opts* opts, mfr_gn_info* info);

/* Twin of mfr_gn_step for HIP graph capture (Sec. 2.3.1, as above), precond 0
 * or 1: the gradient, the CG solve of mfr_pcg_solve_async and armijo_max line
 * search trials are enqueued as one fixed sequence; the Armijo test runs on the
 * device, the trials after an accepted one do nothing, and u is replaced by
 * the accepted point on the device.  u and info equal those of mfr_gn_step bit
 * for bit.  info: device double[9] = {J_before, J_after, eta, slope,
 * pcg_iters, pcg_relres, pcg_flag, accepted, ls_trials} (the fields of
 * mfr_gn_info in order).  A captured graph uses the context's workspace
 * (replay it on the context's stream).  Asynchronous. */
mfr_status mfr_gn_step_async(mfr_ctx* ctx, float* u, const mfr_gn_opts* opts, double* info);

typedef struct mfr_pc mfr_pc;   /* learned preconditioner (see below) */

typedef struct {
  int32_t levels;      /* pyramid levels, 1..8                                     */
  int32_t gn_iters;    /* Gauss-Newton iterations per level                        */
  int32_t pcg_max;     /* CG iterations per Gauss-Newton step                      */
  double pcg_rtol;     /* CG relative residual tolerance                            */
  double armijo_c1;    /* sufficient-decrease constant (e.g. 1e-4)                  */
  int32_t armijo_max;  /* step halvings before the line search gives up             */
  int32_t precond;     /* 0 none, 1 Jacobi, 2 learned (flexible CG with pc)        */
  const float* u_init; /* device [3][n] displacement on the COARSEST deformation
                          grid (mfr_ml_level_grid level 0) the first level starts
                          from; NULL: u = 0 there                                    */
  mfr_pc* pc;          /* precond 2 (three-dimensional problems): the learned
                          preconditioner, bound to each level's context in turn,
                          so its workspace must fit the finest grid; it is left
                          unbound when the call returns, whatever the outcome
                          (mfr_pc_bind before its next use).  Ignored for precond 0, 1; the batched path
                          takes precond 0, 1 only.                                 */
  int32_t fallback_iters; /* precond 2: CG iterations after which a solve that has
                          not converged continues as Jacobi-PCG (0: never)         */
} mfr_ml_opts;

typedef struct {
  double J_final;          /* objective at the returned u on the finest level         */
  int32_t gn_done[8];      /* accepted Gauss-Newton steps per level (coarsest first)  */
  int32_t pcg_total[8];    /* CG iterations per level                                */
  int32_t status[8];       /* 0, or MFR_ELINESEARCH if that level stopped early       */
  double seconds;          /* wall time of the whole call                             */
  double J_start[8];       /* objective of each level at its starting displacement
                              (u_init or 0 on the coarsest, the prolongated field above) */
  double J_level[8];       /* objective of each level at the displacement it hands on  */
} mfr_ml_report;

/* Bytes of device workspace mfr_register_multilevel needs for `finest`. */
mfr_status mfr_ml_workspace_size(const mfr_grid* finest, int32_t levels, size_t* bytes);

/* Grid of pyramid level `level` (0 = coarsest, levels - 1 = `finest`) of a
 * multilevel registration with `levels` levels: ceil(m/2) image cells and
 * ceil((my-1)/2) deformation cells per coarser level, spacings doubled
 * (Sec. 2.3, coarse-to-fine; the coarse grids themselves are not specified by
 * the paper).  The returned grid states the template grid explicitly (mT, hT
 * never 0, also for the finest level). */
mfr_status mfr_ml_level_grid(const mfr_grid* finest, int32_t levels, int32_t level, mfr_grid* out);

/* Coarse-to-fine Gauss-Newton registration (Sec. 2.3): image pyramid of
 * 2x2x2 means (ceil(m/2) cells, spacing doubled), deformation grids with
 * ceil((my-1)/2) cells per coarser level, Gauss-Newton with (P)CG and Armijo
 * line search on each level, linear prolongation of u to the next level.
 * The coarsest level starts from opts->u_init (NULL: 0).  u: device [3][n]
 * of the finest grid, output only: the registered finest displacement.
 * Synchronises the stream. */
mfr_status mfr_register_multilevel(const mfr_grid* finest, const mfr_ml_opts* opts, void* hip_stream,
                                   void* workspace, size_t ws_bytes, const float* R, const float* T,
                                   float* u, mfr_ml_report* report);

/* One level of the image pyramid (Sec. 2.3): coarse[c][b][a] = mean of the
 * fine voxels (2a + i, 2b + j, 2c + k), i, j, k in {0, 1}, an index past the
 * last fine voxel replaced by the last one (odd sizes).  fine: device
 * [m_z][m_y][m_x] float32 with m = m[0..2] (x, y, z), 1 <= m; coarse: device
 * [ceil(m_z/2)][ceil(m_y/2)][ceil(m_x/2)], must not overlap fine.
 * Asynchronous on hip_stream. */
mfr_status mfr_restrict_image(const int32_t m[3], const float* fine, float* coarse, void* hip_stream);

/* Prolongation of a displacement to a finer deformation grid (Sec. 2.3):
 * per dimension, linear interpolation of the coarse node values at the
 * physical position n hy_fine of each fine node, clamped to the coarse grid's
 * extent.  uc: device [3][n_c], uf: device [3][n_f] (no overlap); work: device
 * buffer of at least mfr_prolong_workspace_size(fine) bytes (the per-axis
 * interpolation tables), 256-byte aligned.  Synchronises the stream. */
mfr_status mfr_prolong_workspace_size(const mfr_grid* fine, size_t* bytes);
mfr_status mfr_prolong(const mfr_grid* coarse, const mfr_grid* fine, const float* uc, float* uf, void* work,
                       size_t work_bytes, void* hip_stream);

/* ---- L-BFGS (Sec. 2.3.2) ------------------------------------------------
 * Limited-memory BFGS on J = D + alpha S from the objective and gradient, with
 * the regulariser's Hessian in the initial matrix:
 *   H_0 = alpha nabla^2 S + gamma I = 2 alpha hbar^y L^T L + gamma I, gamma > 0.
 * H_0 is inverted exactly in the cosine (DCT-II) basis that diagonalises the
 * Neumann Laplacian L.  The direction comes from the two-loop recursion over
 * the last `mem` pairs (s, y) with float64 dot products; a pair is kept only
 * if s^T y > 1e-12 |s| |y|; a non-descent direction clears the memory and
 * restarts from -H_0^{-1} grad J.  Step length: Armijo backtracking from 1.
 * The caller provides a device work buffer (256-byte aligned) of at least
 * mfr_lbfgs_workspace_size bytes for the cosine tables and 8 + 2 mem node
 * vectors; at most 4096 nodes per axis. */
#define MFR_LBFGS_MAX_MEM 64

typedef struct {
  int32_t iters;       /* iterations, >= 0                                       */
  int32_t mem;         /* stored pairs, 1..MFR_LBFGS_MAX_MEM                     */
  double gamma;        /* > 0                                                    */
  double armijo_c1;    /* in [0, 1)                                              */
  int32_t armijo_max;  /* step halvings before the line search fails, >= 1       */
} mfr_lbfgs_opts;

typedef struct {
  int32_t iters;          /* accepted iterations                                 */
  int32_t status;         /* 0, or MFR_ELINESEARCH if a line search failed       */
  int32_t restarts;       /* memory cleared after a non-descent direction        */
  int32_t pairs_skipped;  /* pairs that failed the curvature test                */
  int32_t evals;          /* objective evaluations (gradients included)          */
  double J_initial, J_final;
  double seconds;         /* wall time of the call                               */
} mfr_lbfgs_report;

mfr_status mfr_lbfgs_workspace_size(const mfr_grid* grid, int32_t mem, size_t* bytes);

/* x = H_0^{-1} v (all three components).  x may alias v.  work: at least
 * mfr_lbfgs_workspace_size(grid, 1) bytes; every call copies the cosine tables
 * into it (from host copies the context keeps).  Asynchronous. */
mfr_status mfr_h0_solve(mfr_ctx* ctx, double gamma, const float* v, float* x, void* work, size_t work_bytes);

/* Runs opts->iters L-BFGS iterations from u (updated in place).  Synchronises
 * the stream. */
mfr_status mfr_lbfgs(mfr_ctx* ctx, float* u, const mfr_lbfgs_opts* opts, void* work, size_t work_bytes,
                     mfr_lbfgs_report* report);

/* ---- Batched registration of independent pairs ------------------------------
 * Up to MFR_MAX_BATCH image pairs of different sizes advance together: every
 * phase (voxel-tile kernels, node passes, sums, CG vector updates) is one
 * launch for all pairs; the voxel-tile kernels are persistent (work-groups take
 * tiles of any pair from a shared device counter).  The CG iteration is steered
 * on the device (per-pair convergence flags), so a block of iterations is
 * captured once into a HIP graph and replayed.  Results equal running each pair
 * alone through mfr_register_multilevel, bit for bit.  This is an extension of
 * the paper's single-pair method (Sec. 2.3) for throughput; it is not in the
 * paper. */
#define MFR_MAX_BATCH 12

typedef struct mfr_batch mfr_batch;   /* opaque host-side batch context */

typedef struct {
  double J_final[MFR_MAX_BATCH];     /* objective at the returned u (finest level)         */
  int32_t gn_done[MFR_MAX_BATCH];    /* accepted Gauss-Newton steps, all levels            */
  int32_t pcg_total[MFR_MAX_BATCH];  /* CG iterations, all levels                           */
  int32_t status[MFR_MAX_BATCH];     /* 0, or MFR_ELINESEARCH if a level stopped early     */
  int32_t graph_launches;            /* replays of captured CG graphs                      */
  double seconds;                    /* wall time of the call                              */
} mfr_batch_report;

/* Device workspace for `n` pairs (grids[i]: finest grid of pair i) with
 * `levels` pyramid levels each.  The batched path evaluates NGF only: a grid
 * with distance MFR_DIST_SSD is rejected (MFR_EINVAL) here and in
 * mfr_batch_create. */
mfr_status mfr_batch_workspace_size(int32_t n, const mfr_grid* grids, int32_t levels, size_t* bytes);
/* (The batched path also takes the curvature regulariser only.) */

/* Create a batch bound to `hip_stream` and a caller-owned workspace. */
mfr_status mfr_batch_create(int32_t n, const mfr_grid* grids, int32_t levels, void* hip_stream,
                            void* workspace, size_t ws_bytes, mfr_batch** out);
void mfr_batch_destroy(mfr_batch* b);

/* Bind the images of every pair (host arrays of n device pointers) and build
 * the image pyramids in the workspace. */
mfr_status mfr_batch_set_images(mfr_batch* b, const float* const* R, const float* const* T);

/* q_i = (H_i + alpha nabla^2 S_i) p_i at u_i on the finest grids, every pair in
 * one persistent launch (host arrays of n device pointers).  Asynchronous. */
mfr_status mfr_batch_hess_vec(mfr_batch* b, const float* const* u, const float* const* p, float* const* q);

/* Coarse-to-fine Gauss-Newton registration of every pair (options as in
 * mfr_register_multilevel; opts->levels must equal the batch's levels;
 * opts->u_init must be NULL: every pair starts at u = 0).
 * use_graph != 0 replays the CG iterations from captured HIP graphs.
 * u: host array of n device pointers to the finest displacements (output).
 * Synchronises the stream. */
mfr_status mfr_batch_register(mfr_batch* b, const mfr_ml_opts* opts, int32_t use_graph, float* const* u,
                              mfr_batch_report* report);

/* ---- Learned preconditioner -------------------------------------------------------
 * An extension of the method (the paper solves the Newton equation with plain
 * CG): a 3D CNN on the deformation-node grid maps the CG residual r to a search
 * direction z for flexible CG,
 *   y = r / diag (Jacobi),  z = y + rms(y) * CNN(features)[0..2],
 * features per node = RMS-normalised y (3), r (3), diag (3) and |grad R| (1,
 * the voxel gradient magnitude of R averaged onto the nodes with the weights of
 * the grid conversion, eq. grid_conversion), zero-padded to 16 channels.
 * Network: four 3x3x3 convolutions 16 -> 16 channels, zero padding, ReLU after
 * the first three; bf16 weights and activations with fp32 accumulation on the
 * matrix cores; the last layer's outputs 3..15 are unused (held at zero).
 * Parameters (fp32 master copy): per layer [27 taps][16 in][16 out] weights,
 * tap t = 9 (dz+1) + 3 (dy+1) + (dx+1), then 16 biases. */
#define MFR_PC_PARAMS (4 * (27 * 16 * 16 + 16))

/* mfr_pc (opaque, bound to one context: grid, stream, images) is declared before mfr_ml_opts. */

/* Device workspace of a preconditioner for `grid`; train != 0 adds the
 * gradient, optimiser and backward buffers. */
mfr_status mfr_pc_workspace_size(const mfr_grid* grid, int32_t train, size_t* bytes);
/* Create on ctx's stream (parameters zero: z = y until mfr_pc_set_params).
 * The context must have images; |grad R| is recomputed when they change. */
mfr_status mfr_pc_create(mfr_ctx* ctx, int32_t train, void* workspace, size_t ws_bytes, mfr_pc** out);
void mfr_pc_destroy(mfr_pc* pc);
/* Rebind to another context (another grid size; the network parameters and
 * optimiser state are kept).  The workspace must be large enough for that
 * context's grid (MFR_ENOMEM otherwise).  Detaches the preconditioner from its
 * previous context. */
mfr_status mfr_pc_bind(mfr_pc* pc, mfr_ctx* ctx);
/* Copy MFR_PC_PARAMS floats from / to host memory (synchronous). */
mfr_status mfr_pc_set_params(mfr_pc* pc, const float* params);
mfr_status mfr_pc_get_params(mfr_pc* pc, float* params);
/* z = M(r) with the Jacobi diagonal taken at u (device [3][n] vectors). */
mfr_status mfr_pc_apply(mfr_pc* pc, const float* u, const float* r, float* z);

typedef struct {
  double lr, beta1, beta2, eps;   /* Adam                                          */
  int32_t pcg_iters;              /* Jacobi-PCG iterations run on the system       */
  int32_t sample_every;           /* one training step on every k-th residual      */
} mfr_pc_train_opts;

typedef struct {
  int32_t steps;                  /* training steps taken                          */
  double loss_first, loss_last, loss_mean;
} mfr_pc_train_info;

/* Train on one Gauss-Newton system (H + alpha nabla^2 S) s = b at u: run
 * Jacobi-PCG on it and take an Adam step on every sample_every-th residual r.
 * Loss per residual: L = -((z.r)^2 / z.Az) / ((y.r)^2 / y.Ay), the energy
 * decrease of the best step along z relative to the Jacobi direction y
 * (-1 for z = y; lower is better); dL/dz = 2s(s Az - r)/E_J with s = z.r/z.Az.
 * Needs a preconditioner created with train != 0.  Synchronises. */
mfr_status mfr_pc_train_system(mfr_pc* pc, const float* u, const float* b, const mfr_pc_train_opts* opts,
                               mfr_pc_train_info* info);

/* Attach (or detach with NULL) the preconditioner used by precond = 2. */
mfr_status mfr_attach_pc(mfr_ctx* ctx, mfr_pc* pc);

/* The convolution kernels themselves, for testing and reuse: node grid nx x ny
 * x nz, activations [z][y][x][16] bf16 (raw 16-bit patterns), weights
 * [27][16][16] bf16, bias fp32[16] (nullable).  Asynchronous on `hip_stream`.
 * mfr_cnn_conv: y = conv(x) + bias, ReLU if relu != 0; outputs y32 (fp32
 * [n][16]) and/or y16 (bf16 [n][16]), either may be NULL.
 * mfr_cnn_conv_bwd_data: dx = conv^T(g) (the gradient with respect to the
 * input), zeroed where mask <= 0 (mask: the bf16 input activations, nullable).
 * mfr_cnn_conv_bwd_weight: dwb = [dW (27*16*16) | db (16)] fp32 of sum(g * y)
 * with respect to the weights and bias, with a device workspace of
 * mfr_cnn_wgrad_workspace_size bytes. */
mfr_status mfr_cnn_conv(int32_t nx, int32_t ny, int32_t nz, const uint16_t* x, const uint16_t* w,
                        const float* bias, int32_t relu, float* y32, uint16_t* y16, void* hip_stream);
mfr_status mfr_cnn_conv_bwd_data(int32_t nx, int32_t ny, int32_t nz, const uint16_t* g, const uint16_t* w,
                                 const uint16_t* mask, float* dx32, uint16_t* dx16, void* hip_stream);
mfr_status mfr_cnn_wgrad_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t* bytes);
mfr_status mfr_cnn_conv_bwd_weight(int32_t nx, int32_t ny, int32_t nz, const uint16_t* x, const uint16_t* g,
                                   float* dwb, void* workspace, size_t ws_bytes, void* hip_stream);

/* ---- Tile configuration ---------------------------------------------------------
 * Shape of the voxel-tile work-groups (bx x by threads: 32x16, 64x8, 32x32 or
 * 64x16), the number of z planes per group (chunk_len; 0 = derived from
 * target_groups) and the number of work-groups the derived split aims for
 * (target_groups; 0 = 2048), for contexts and batches created afterwards in
 * this process.  Returns MFR_EINVAL for an unsupported shape or a negative
 * count.  The tile autotuner sets it from measured timings. */
typedef struct {
  int32_t bx, by, chunk_len, target_groups;
} mfr_tile_config;

mfr_status mfr_set_tile_config(const mfr_tile_config* cfg);
mfr_status mfr_get_tile_config(mfr_tile_config* cfg);

/* Kernel timing for measurement.  While enabled, the library records a pair
 * of HIP events on the context's stream around every launch of its main
 * kernels; mfr_profile_read synchronises the stream and returns the launch
 * counts and summed event times in milliseconds, per kernel:
 * [0] voxel-tile kernel, objective mode; [1] gradient mode; [2] Hessian-vector
 * mode; [3] Jacobi diagonal; [4] node pass (all modes); [5] the attached or
 * applied learned preconditioner's network (its features and four
 * convolutions, one record per application).  Timing adds two event records
 * per launch; it is off after mfr_create. */
typedef struct {
  int32_t launches[6];
  double ms[6];
} mfr_profile_stats;

mfr_status mfr_profile_enable(mfr_ctx* ctx, int32_t enable);
mfr_status mfr_profile_read(mfr_ctx* ctx, mfr_profile_stats* stats, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* MFR_H */
