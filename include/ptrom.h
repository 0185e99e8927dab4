/*
 * ptrom.h - C ABI of libptrom: the regularized 2D Biot-Savart pair sum, its
 * Jacobian products and adjoint, explicit and implicit time steppers, a
 * batched multi-instance stepper, a checkpointed RK4 adjoint, and the online
 * step of the projection-tree reduced-order model (PTROM) of
 * Rodriguez et al., "Projection-tree reduced order modeling for fast N-body
 * computations" (arXiv 2103.01983), on AMD MI355X (gfx950).
 *
 * Notation follows the paper:
 *   N bodies with positions chi_i (x) and psi_i (y) and circulations Gamma_i.
 *   State vector layout (problem formulation, state-vector definition):
 *       xy[0..N) = x_0..x_{N-1},  xy[N..2N) = y_0..y_{N-1}     ("SoA")
 *   Velocity (kernel equation; target-source form f = K gamma):
 *       f_i = sum_{j != i} Gamma_j / (2 pi) * (-r_y, r_x) / (|r|^2 + delta^2),
 *       r = x_i - x_j  (target minus source).
 *   delta is the de-singularisation core; it enters squared (delta is a
 *   length).  delta = 0 is legal: self pairs are excluded by index, but two
 *   distinct coincident bodies then give non-finite values (not checked).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers owned by the caller unless the
 *     comment says "host".  The library never keeps a caller pointer after
 *     the call returns (ptrom_rom_create copies what it needs).
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *     = the null stream) unless documented as synchronising.
 *   - A context owns a grow-only device workspace; calls made through one
 *     context must not run concurrently (use one context per stream/thread).
 *   - Return value: PTROM_OK (0) on success; PTROM_ENOCONV (1) is a warning
 *     (an iteration cap was hit, results are still written); negative values
 *     are errors, with a message from ptrom_last_error().  Arguments are
 *     validated before anything is launched: N >= 1 and N <= 2^30,
 *     delta >= 0, dt > 0, nsteps >= 0, non-NULL required pointers, else
 *     PTROM_EINVAL and nothing is written.
 */
#ifndef PTROM_H
#define PTROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptrom_ctx ptrom_ctx;
typedef struct ptrom_rom ptrom_rom;
typedef void *ptrom_stream; /* hipStream_t */

enum {
  PTROM_OK = 0,
  PTROM_ENOCONV = 1,
  PTROM_EINVAL = -1,
  PTROM_ENOMEM = -2,
  PTROM_EHIP = -3
};

/* Implicit one-step schemes of the linear multistep residual (eq. "linKstep"
 * with k = 1): backward Euler (alpha0 = 1, alpha1 = -1, beta0 = 1,
 * beta1 = 0) and the trapezoid rule the paper uses (beta0 = beta1 = 1/2). */
enum { PTROM_BACKWARD_EULER = 0, PTROM_TRAPEZOID = 1 };

/* HyperPair Jacobian: PAPER = the paper's inexact Jacobian (only the 2x2
 * derivative of each sampled velocity with respect to its own target
 * position, Section "Problem formulation" and Algorithm "HyperPair");
 * EXACT = also differentiates the surrogate-source positions. */
enum { PTROM_JAC_PAPER = 0, PTROM_JAC_EXACT = 1 };

/* Library version (major*10000 + minor*100 + patch). */
int ptrom_version(void);

/* Create a context bound to HIP device `device`; loads tuned launch
 * parameters from the file named by the environment variable
 * PTROM_TUNE_CACHE if it exists.  *out is set only on success. */
int ptrom_create(ptrom_ctx **out, int device);
/* Free a context and its workspace (synchronises the device). NULL is a no-op. */
void ptrom_destroy(ptrom_ctx *ctx);
/* Message of the last error on this context ("" if none). The pointer stays
 * valid until the next call on the context. */
const char *ptrom_last_error(const ptrom_ctx *ctx);

/* ------------------------------------------------------------------------
 * Pair sums (kernel equation and its derivatives).  FP32 arithmetic with
 * two-level compensated (Kahan) accumulation over sources.
 * ---------------------------------------------------------------------- */

/* f[2N] = velocity of every body (SoA). Kernel equation ("BS_kernel"). */
int ptrom_velocity(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
                   float *f, ptrom_stream stream);

/* ptrom_velocity for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments and result, but the call allocates nothing.  Partial sums
 * go to a fixed 36 MiB device array that the library holds on every device
 * it runs on until the process ends (its address is looked up once per
 * device by ptrom_create).  The launch is the context's own when its
 * workspace fits that array (N <= 32768 with the shipped table: results
 * bitwise equal to ptrom_velocity's); beyond, the one-sided pair kernel with
 * as many source chunks as fit (the same FP32 sums in another order; above
 * 2.36 million bodies one chunk, which needs no scratch).  A launch needing
 * more than the array is rejected with PTROM_ENOMEM and a message (it cannot
 * arise with these rules).  All calls on one device share the array, so
 * calls that overlap on one device (other streams, other threads or
 * contexts) race; serialise them.  Errors as ptrom_velocity; PTROM_EHIP if
 * the array's address could not be looked up. */
int ptrom_velocity_noalloc(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
                           float *f, ptrom_stream stream);

/* FP64 version of ptrom_velocity (plain double sums, IEEE division). */
int ptrom_velocity_f64(ptrom_ctx *ctx, int64_t n, const double *xy, const double *gamma,
                       double delta, double *f, ptrom_stream stream);

/* Jacobian-vector product jv = (df/dx) v, v and jv [2N] SoA:
 *   (Jv)_i = sum_{j != i} Gamma_j/(2pi) H(r_ij) (v_i - v_j),
 *   H(r) = d/dr[(-r_y, r_x)/s] = (1/s^2) [[2 r_x r_y, r_y^2 - r_x^2 - delta^2],
 *                                         [r_y^2 - r_x^2 + delta^2, -2 r_x r_y]],
 *   s = |r|^2 + delta^2.  Used by implicit (LSPG/Newton) residual Jacobians
 *   (Section "Least-Squares Petrov-Galerkin projection"). */
int ptrom_jvp(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
              const float *v, float *jv, ptrom_stream stream);

/* Per-body 2x2 self blocks B_i = sum_{j != i} Gamma_j/(2pi) H(r_ij), the
 * paper's inexact "diagonal block" kernel Jacobian (problem formulation).
 * Output B[4][N]: B00, B01, B10, B11 planes (B11 = -B00). */
int ptrom_block_jacobian(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                         float delta, float *B, ptrom_stream stream);

/* Velocity f[2N] (as ptrom_velocity) and the self blocks B[4N] (as
 * ptrom_block_jacobian) in one pass over the pairs: both need the same
 * separation and reciprocal per pair, and the paper's inexact Newton needs
 * both at every iterate (problem formulation, after eq. "linKstep"). */
int ptrom_velocity_block_jacobian(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                                  float delta, float *f, float *B, ptrom_stream stream);

/* Adjoint (vector-Jacobian product) for a cotangent w [2N]:
 *   gxy[2N]    = (df/dx)^T w,  (J^T w)_k = sum_{j != k} H(r_kj)^T (G_j w_k - G_k w_j)/(2pi)
 *   ggamma[N]  = d(w.f)/dGamma_k = (1/2pi) sum_{i != k} w_i . (-r_y, r_x)/s, r = x_i - x_k. */
int ptrom_vjp(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
              const float *w, float *gxy, float *ggamma, ptrom_stream stream);

/* Stream function of the regularized flow at every body, induced by the
 * others: psi_i = -(1/4pi) sum_{j != i} Gamma_j log(|r|^2 + delta^2); psi[N].
 * The Hamiltonian of the metrics section (in its regularized, conserved form)
 * is H = 1/2 sum_i Gamma_i psi_i, and f_i = (d psi_i/dy_i, -d psi_i/dx_i). */
int ptrom_stream_function(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
                          float *psi, ptrom_stream stream);

/* The Hamiltonian of the metrics section in its regularized, conserved form,
 *   H = -(1/4pi) sum_{i != j} Gamma_i Gamma_j 1/2 log(|r_ij|^2 + delta^2)
 *     = 1/2 sum_i Gamma_i psi_i   (psi as in ptrom_stream_function),
 * written to H (DEVICE, one double).  The stream function is summed in FP32
 * (compensated), the final sum over bodies in FP64 in a fixed order.  The
 * paper's printed form is its delta = 0 case with the opposite sign. */
int ptrom_hamiltonian(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta, double *H,
                      ptrom_stream stream);

/* Velocity induced at nt arbitrary points p [2][nt] (SoA) by all n bodies, no
 * exclusion (the grid velocity field of the metrics section); f [2][nt]. */
int ptrom_velocity_points(ptrom_ctx *ctx, int64_t nt, const float *p, int64_t n, const float *xy,
                          const float *gamma, float delta, float *f, ptrom_stream stream);

/* ------------------------------------------------------------------------
 * Time steppers.
 * ---------------------------------------------------------------------- */

/* nsteps classic RK4 steps of dx/dt = f(x) in place on xy[2N]. */
int ptrom_rk4(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta, float dt,
              int nsteps, ptrom_stream stream);

/* FP64 RK4 (uses ptrom_velocity_f64). */
int ptrom_rk4_f64(ptrom_ctx *ctx, int64_t n, double *xy, const double *gamma, double delta,
                  double dt, int nsteps, ptrom_stream stream);

/* Linear model of each Newton correction (ptrom_newton_opts.linear_solver):
 * GMRES = the exact Jacobian, applied through Jacobian-vector products and
 * solved by restarted GMRES; BLOCK = the paper's inexact Jacobian, which
 * keeps only each body's own 2x2 block df_i/dx_i (Section "Problem
 * formulation", after eq. "linKstep"), solved body by body. */
enum { PTROM_NEWTON_GMRES = 0, PTROM_NEWTON_BLOCK = 1 };

typedef struct {
  double newton_tol;  /* stop when |r(xi)| <= newton_tol * |r(x_prev)| (default 1e-6) */
  int32_t max_newton; /* Newton iterations per step (default 20) */
  int32_t gmres_restart; /* GMRES: Krylov basis size, 1 to 200 (default 20) */
  int32_t gmres_maxit;   /* GMRES: matvecs per Newton iteration (default 60) */
  int32_t linear_solver; /* PTROM_NEWTON_GMRES (default) or PTROM_NEWTON_BLOCK */
  double gmres_tol;   /* GMRES: relative residual of each Newton linear solve (default 1e-3) */
  int32_t jac_period; /* BLOCK: 0 = blocks evaluated at every Newton iterate; p >= 1 =
                         evaluated at the first iterate (x_prev) of steps 0, p, 2p, ...
                         of the call and kept in between (default 0) */
  int32_t pad;
} ptrom_newton_opts;

typedef struct {
  int32_t newton_iters; /* total over all steps */
  int32_t krylov_iters; /* total Jacobian products (0 with PTROM_NEWTON_BLOCK) */
  int32_t nonconverged_steps;
  int32_t pad;
  double max_final_rel_residual; /* max over steps of |r_final| / |r_0| */
} ptrom_newton_stats;

/* nsteps implicit steps (scheme = PTROM_BACKWARD_EULER or PTROM_TRAPEZOID) of
 * the k=1 linear multistep residual, each solved by Newton's method whose
 * linear systems (I - dt beta0 J) d = -r are solved matrix-free by restarted
 * GMRES over ptrom_jvp, or, with linear_solver = PTROM_NEWTON_BLOCK, with J
 * replaced by the per-body blocks of ptrom_block_jacobian (2x2 solves; a
 * singular block gives non-finite output and PTROM_ENOCONV).  The unknown
 * is the increment xi - x_prev.  opts may be NULL (defaults).  stats may be
 * NULL.  SYNCHRONISES the stream (host-side Newton and Krylov scalars).
 * Returns PTROM_ENOCONV if a step hit max_newton. */
int ptrom_implicit(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta,
                   float dt, int nsteps, int scheme, const ptrom_newton_opts *opts,
                   ptrom_newton_stats *stats, ptrom_stream stream);

/* Same with a background velocity uinf [2N] (device, SoA; may be NULL) added
 * to every body's right-hand side, dx_i/dt = f_i(x) + uinf_i: the inflow
 * condition of the mushroom-cloud parametric experiment.  It enters the
 * residual as - dt (beta0 + beta1) uinf; the Jacobian is unchanged. */
int ptrom_implicit_forced(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta,
                          const float *uinf, float dt, int nsteps, int scheme, const ptrom_newton_opts *opts,
                          ptrom_newton_stats *stats, ptrom_stream stream);

/* ------------------------------------------------------------------------
 * Batched parametric instances: nb independent systems in one persistent
 * launch per velocity evaluation.
 *   offsets (host) [nb+1]: instance b owns bodies offsets[b]..offsets[b+1]-1;
 *   xy: instance b's SoA block [x..., y...] occupies xy[2*offsets[b] .. 2*offsets[b+1]);
 *   gamma[offsets[nb]]; delta (host) [nb] per-instance cores.
 * Every unordered pair of an instance is evaluated once, in blocks of 256 K
 * bodies, K targets per lane (1, 2 or 4) and the workgroups per CU taken from
 * the tuning table's "batched_velocity" entry for the instance set's
 * pair-weighted mean size sum N_b^2 / sum N_b (ptrom_autotune measures it;
 * default K = 2, 8 per CU).  The workspace holds one slot per block and body:
 * 8 * sum_b ceil(N_b / (256 K)) * N_b bytes.  EINVAL when the instances hold
 * more than 2^24 block pairs in total or the slots would pass 1/32 of the
 * device's memory.
 * ---------------------------------------------------------------------- */
int ptrom_velocity_batched(ptrom_ctx *ctx, int nb, const int64_t *offsets, const float *xy,
                           const float *gamma, const float *delta, float *f, ptrom_stream stream);

/* nsteps RK4 steps for every instance, captured once into a HIP graph and
 * replayed (use_graph = 0 launches the same kernels directly). */
int ptrom_rk4_batched(ptrom_ctx *ctx, int nb, const int64_t *offsets, float *xy,
                      const float *gamma, const float *delta, float dt, int nsteps,
                      int use_graph, ptrom_stream stream);

/* ------------------------------------------------------------------------
 * Discrete RK4 adjoint with step checkpointing.
 * ---------------------------------------------------------------------- */

/* Forward: nsteps RK4 steps from xy0; stores the state at steps
 * 0, every, 2*every, ... into ckpt[ceil(nsteps/every)][2N] and x(T) in xyT. */
int ptrom_rk4_fwd_ckpt(ptrom_ctx *ctx, int64_t n, const float *xy0, const float *gamma,
                       float delta, float dt, int nsteps, int every, float *ckpt, float *xyT,
                       ptrom_stream stream);

/* Backward: given lamT = dQ/dx(T) [2N] and optionally the direct partial
 * ggamma_direct = dQ/dGamma at fixed x(T) [N] (may be NULL), writes
 * lam0 = dQ/dx(0) [2N] and ggamma = total dQ/dGamma [N] for the discrete RK4
 * map, recomputing each segment's stage inputs from its checkpoint. */
int ptrom_rk4_bwd(ptrom_ctx *ctx, int64_t n, const float *ckpt, const float *gamma, float delta,
                  float dt, int nsteps, int every, const float *lamT, const float *ggamma_direct,
                  float *lam0, float *ggamma, ptrom_stream stream);

/* ------------------------------------------------------------------------
 * Online PTROM (Algorithms "Gauss-Newton" and "HyperPair").
 * ---------------------------------------------------------------------- */

/* Offline artifacts, all HOST arrays (copied by ptrom_rom_create).
 * Sampled rows are ordered [chi of the ns sampled bodies, psi of them]. */
typedef struct {
  int32_t M;        /* state POD rank */
  int32_t Mr;       /* residual POD rank (rows of A) */
  int32_t ns;       /* sampled bodies; nd = 2*ns sampled rows */
  int32_t jac_mode; /* PTROM_JAC_PAPER or PTROM_JAC_EXACT */
  int64_t Nc;       /* unique surrogate sources (clusters and single bodies) */
  int64_t nnz;      /* total entries of the interaction lists */
  const double *Phibar; /* [nd][M]  rows of Phi at the sampled rows */
  const double *xbar0;  /* [nd]     x^0 at the sampled rows */
  const double *xqt0;   /* [Nc][2]  surrogate reference positions */
  const double *Phit;   /* [Nc][2][M] surrogate POD rows (Phi tilde) */
  const double *Gt;     /* [Nc]     surrogate circulations (Gamma tilde) */
  const int64_t *off;   /* [ns+1]   CSR offsets of each sampled target's list */
  const int64_t *ids;   /* [nnz]    surrogate ids in [0, Nc); a target's own body never appears */
  const double *A;      /* [Mr][nd] gappy operator [P Phi_r]^+ */
  double delta, dt;
  double tol;           /* relative reduced-gradient tolerance */
  double alpha;         /* Gauss-Newton step length (the paper uses 1) */
  int32_t max_iter;     /* Gauss-Newton iterations per step (the paper caps at 100) */
  int32_t pad;
  const double *ubar;   /* [nd] background velocity at the sampled rows (the
                           mushroom cloud's inflow), or NULL for none; it is
                           part of the sampled velocity fbar and so of the
                           trapezoid residual rows */
} ptrom_rom_desc;

/* Copy the artifacts to the device (surrogate and sampled rows as FP32 for
 * the gather, A as FP64 for the least-squares solve).  Requires
 * 1 <= M <= 112, M <= Mr <= 256, 1 <= ns <= 2^20, ids in [0, Nc); the exact
 * Jacobian needs M <= 32 and Mr <= 64.  Bases beyond 32 / 64 take a blocked
 * path whose per-query arrays must fit one workgroup's LDS (EINVAL from the
 * run calls otherwise). */
int ptrom_rom_create(ptrom_ctx *ctx, const ptrom_rom_desc *desc, ptrom_rom **out);
void ptrom_rom_destroy(ptrom_rom *rom);

/* One HyperPair evaluation at xhat (device FP64 [M]) with previous-step
 * terms xbar_prev, fbar_prev (device FP64 [nd]); writes sampled positions
 * xbar, velocities fbar, trapezoid residual rows rbar ([nd] FP64) and the
 * residual Jacobian times Phibar, C ([nd][M] FP64).  Any output may be NULL. */
int ptrom_rom_hyperpair(ptrom_rom *rom, const double *xhat, const double *xbar_prev,
                        const double *fbar_prev, double *xbar, double *fbar, double *rbar,
                        double *C, ptrom_stream stream);

/* nsteps online time steps in one device-resident launch (one workgroup, or
 * for long lists several, see ptrom_rom_set_split), starting from xhat
 * (device FP64 [M], updated in place).  Per step:
 * Gauss-Newton iterations (Algorithm "Gauss-Newton") of HyperPair + the FP64
 * least-squares step dxhat = -argmin |A C nu + A rbar|, solved through the
 * normal equations (AC)^T (AC) by Gauss-Jordan elimination with one
 * refinement on the true residual (M <= 32, M_r <= 64), or for larger bases
 * by blocked Gauss-Jordan inversion of the normal matrix (C held in FP32
 * there; positions, separations and residual in FP64), xhat += alpha dxhat,
 * until the relative reduced gradient |(AC)^T A rbar| / (its first-iteration
 * value) <= tol or max_iter iterations.  A direction with a non-positive
 * pivot is left out of the step.  xhat_hist (device [nsteps][M]) and iters
 * (device int32 [nsteps]) may be NULL.  EINVAL when a larger basis's arrays
 * do not fit one workgroup's LDS.  Asynchronous; iteration caps are reported
 * in iters only. */
int ptrom_rom_run(ptrom_rom *rom, int nsteps, double *xhat, double *xhat_hist, int32_t *iters,
                  ptrom_stream stream);

/* Workgroups per query of the small-basis runs with the paper's Jacobian
 * (ptrom_rom_run, ptrom_rom_run_batched; M <= 32, M_r <= 64, arrays in LDS).
 * With W > 1 each of a query's W workgroups keeps a contiguous slice of the
 * interaction-list entries in LDS and sums its slice's HyperPair terms per
 * target; the W partial sums meet at a device-side counter barrier once per
 * HyperPair evaluation and are added in slice order, and every workgroup then
 * runs the same least-squares step, so all of them hold the same xhat.  The
 * launch is cooperative (all W x nq workgroups resident).  workgroups: 0 =
 * automatic (about 1024 entries per slice, at most 16, widened until a slice
 * fits in LDS; no split below 4096 entries), 1 = one workgroup per
 * query, 2..64 = that many (widened if a slice does not fit).  The split is
 * skipped, silently, where the device takes no cooperative launch or the grid
 * would not be resident at once.  A barrier wait that fails max_polls checks
 * (0: the default, 2^20 checks, about a second, which a resident grid never
 * reaches; a small value forces the path) stops every workgroup of the
 * launch at its next barrier and reports iters = -1 for every step of each
 * affected query and a NaN xhat.  Calls on one context share its workspace,
 * which holds the partial sums and counters; runs that overlap on one
 * context race.  EINVAL for workgroups outside 0..64. */
int ptrom_rom_set_split(ptrom_rom *rom, int workgroups, uint32_t max_polls);

/* The workgroups per query (1 = no split) that ptrom_rom_run (batched_nq = 0)
 * or ptrom_rom_run_batched with batched_nq queries would use for nsteps
 * steps, written to *workgroups (host int32).  Launches nothing.  EINVAL for
 * a NULL output or negative counts. */
int ptrom_rom_split_plan(ptrom_rom *rom, int batched_nq, int nsteps, int32_t *workgroups);

/* Parametric queries (online computations: the tree keeps the bodies of each
 * cluster, so the clustered circulations are reloaded for a new parameter
 * without retraining).
 *
 * ptrom_rom_members: the bodies of each surrogate, HOST CSR arrays mem_off
 * [Nc+1] (mem_off[0] = 0, every surrogate non-empty) and mem_ids (body ids in
 * [0, n)), as from ptrom_cluster_members; copied to the device.  SYNCHRONISES
 * when it replaces an earlier membership.
 *
 * ptrom_rom_reassign: Gamma~_q[c] = sum over the members j of c of
 * gamma_q[q][j], for nq queries; gamma_q device FP32 [nq][n], gt_q device FP32
 * [nq][Nc] (sums accumulated in FP64).  Asynchronous.
 *
 * ptrom_rom_run_batched: nq independent online runs in one launch, one
 * workgroup per query (or several, as for ptrom_rom_run), query q using the circulations gt_q[q] (device FP32
 * [nq][Nc]) and its own xhat[q] (device FP64 [nq][M], in place), xhat_hist
 * [nq][nsteps][M] and iters [nq][nsteps] (both may be NULL).  Surrogate
 * positions and rows are those of the artifacts.  EINVAL when the run arrays
 * of one query do not fit in a workgroup's LDS.  Asynchronous. */
int ptrom_rom_members(ptrom_rom *rom, int64_t n, const int64_t *mem_off, const int64_t *mem_ids);
int ptrom_rom_reassign(ptrom_rom *rom, int nq, const float *gamma_q, float *gt_q, ptrom_stream stream);
int ptrom_rom_run_batched(ptrom_rom *rom, int nq, const float *gt_q, int nsteps, double *xhat,
                          double *xhat_hist, int32_t *iters, ptrom_stream stream);

/* ------------------------------------------------------------------------
 * Offline training helpers (training hierarchy, Stages 2-3).
 * ---------------------------------------------------------------------- */

typedef struct ptrom_clusters ptrom_clusters;

/* Host-side (no GPU) quadtree over the weighted POD points and per-target
 * source clustering (Algorithms "ClusterPOD" and "checkPrune").
 * All arrays are HOST memory:
 *   wpts [n][2]  each body's point in W_phi = Phi Sigma_hat ((Phi s)_i, (Phi s)_{i+n});
 *   xy0 [2n]     reference state x^0 (SoA);  phi [2n][M] POD basis, row-major;
 *   gamma [n];   max_level = depth cap of the tree (root = level 0);
 *   criterion    0 = neighbour search: prune a source cell that does not
 *                overlap the target leaf grown by pc times its width (Def. 2;
 *                pc >= 0, INFINITY prunes nothing);
 *                1 = Barnes-Hut: prune when w / |s - s_i| <= theta, w the cell
 *                width, s its |Gamma|-weighted mean point, s_i the target's
 *                point (theta >= 0; 0 prunes nothing but zero-width cells);
 *   targets [nt] body ids whose interaction lists are built.
 * Readings of the open passages: root = tight bounding box; midpoint splits
 * while a cell holds > 1 body and is above max_level; half-open membership;
 * width = longer side; |Gamma|-weighted means, strength = sum of Gamma; a
 * cell holding the target is never pruned; an unpruned leaf expands into its
 * bodies minus the target.  Unique surrogates: single bodies first (by id),
 * then cells (by level, row, column); every list is sorted by surrogate id.
 * The result object owns its arrays; read them with ptrom_cluster_fetch. */
int ptrom_cluster_build(int64_t n, const double *wpts, const double *xy0, const double *phi, int M,
                        const double *gamma, int max_level, int criterion, double pc, double theta,
                        int64_t nt, const int64_t *targets, ptrom_clusters **out);
int ptrom_cluster_sizes(const ptrom_clusters *c, int64_t *nc, int64_t *nnz);
/* Copies into caller HOST buffers (any may be NULL): xqt0 [Nc][2], phit
 * [Nc][2][M], gt [Nc], off [nt+1], ids [nnz], keys [Nc] (body id, or
 * 2^60 | level<<40 | row<<20 | column for a cell). */
int ptrom_cluster_fetch(const ptrom_clusters *c, double *xqt0, double *phit, double *gt, int64_t *off,
                        int64_t *ids, int64_t *keys);
void ptrom_cluster_destroy(ptrom_clusters *c);

/* The bodies each unique surrogate stands for, in surrogate order (the body
 * itself, or every body of the cell in increasing id order): CSR arrays in
 * caller HOST memory, mem_off [Nc+1] and mem_ids [*nmem].  *nmem is always
 * written; either array may be NULL (call once with NULLs to size them).
 * Online computations reassign clustered circulations for a new parameter
 * from this membership. */
int ptrom_cluster_members(const ptrom_clusters *c, int64_t *nmem, int64_t *mem_off, int64_t *mem_ids);

/* FP64 Gram matrix G = X X^T of k device rows X [k][nd] (row-major);
 * G [k][k] device.  Used for the POD by the method of snapshots. */
int ptrom_gram_f64(ptrom_ctx *ctx, int64_t nd, int k, const double *X, double *G, ptrom_stream stream);

/* FP64 combination Y = T^T X: Y [M][nd] = sum_a T[a][m] X[a][q] with X [k][nd],
 * T [k][M] (device).  Forms the basis from snapshots and applies R^{-1} in
 * the CholeskyQR re-orthogonalisation. */
int ptrom_combine_f64(ptrom_ctx *ctx, int64_t nd, int k, const double *X, int M, const double *T,
                      double *Y, ptrom_stream stream);

/* ------------------------------------------------------------------------
 * Launch-parameter autotuning.
 * ---------------------------------------------------------------------- */

/* Time the candidate launch configurations of the pair kernels on this
 * device at a set of sizes, keep the fastest per (operation, size class) in
 * the context and, if cache_path is not NULL, write them there (text).
 * The batched velocity launch is tuned too, on instance sets of equal sizes
 * 2048, 8192 and 32768.
 * SYNCHRONISES; allocates temporary device buffers. */
int ptrom_autotune(ptrom_ctx *ctx, const char *cache_path);

/* Load tuned parameters written by ptrom_autotune. */
int ptrom_load_tuning(ptrom_ctx *ctx, const char *cache_path);

/* Pair-kernel operations, as named in the tuning file. */
enum {
  PTROM_OP_VELOCITY = 0,
  PTROM_OP_BLOCK_JACOBIAN = 1,
  PTROM_OP_JVP = 2,
  PTROM_OP_VJP = 3,
  PTROM_OP_STREAM_FUNCTION = 4,
  PTROM_OP_VELOCITY_BLOCK_JACOBIAN = 5,
  PTROM_OP_BATCHED_VELOCITY = 6 /* ptrom_pair_config only: the batched launch for
                                   instance sets whose pair-weighted mean size
                                   sum N_b^2 / sum N_b is n (out[1] targets per
                                   lane, out[2] workgroups per CU) */
};

/* The launch the context would use for operation op at n bodies, written to
 * the caller's HOST array out[5]: source staging (0 LDS tiles, 1 scalar
 * cache), targets per lane, waves per SIMD, each-unordered-pair-once form
 * (0/1), and the number of source chunks of the one-sided form
 * (0 for the each-pair-once form).  The each-pair-once form keeps one
 * partial-sum slot per body and block of 256 K bodies, a workspace that grows
 * as N^2; where it would pass 1/32 of the device's memory the one-sided form
 * (workspace O(N)) is used instead.  Host only; EINVAL for an unknown op or n
 * outside [1, 2^30]. */
int ptrom_pair_config(ptrom_ctx *ctx, int op, int64_t n, int32_t *out);

/* The same decision without a device or context (capacity planning; uses no
 * HIP call): the launch a device with num_cus compute units and device_bytes
 * of memory would use for op at n bodies under the tuning file tuning_path
 * (NULL: the built-in defaults), written to out[5] as above, and the
 * workspace in bytes that launch needs (ws_bytes may be NULL).  EINVAL for an
 * unknown op, n outside [1, 2^30], num_cus < 1, device_bytes = 0, or a
 * tuning file that cannot be read or holds no entries. */
int ptrom_pair_plan(const char *tuning_path, int num_cus, uint64_t device_bytes, int op, int64_t n,
                    int32_t *out, uint64_t *ws_bytes);

#ifdef __cplusplus
}
#endif

#endif /* PTROM_H */
