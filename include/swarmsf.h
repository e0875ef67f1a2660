/*
 * swarmsf.h -- C ABI of the batched Swarm-Gen safety filter (SF) for MI355X (gfx950).
 *
 * The SF projects sampled joint swarm trajectories onto the set of trajectories that
 * satisfy the boundary conditions (eq. boundary_con), pairwise collision avoidance
 * (eq. inter_robot_con) and velocity/acceleration bounds, with the fixed-point
 * iteration of the Appendix ("Custom SF optimizer", eqs. alpha_step .. xi_step):
 * per-pair/per-time projections, the multiplier step, and an equality-constrained
 * QP step against a factorisation computed once by sf_setup.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers unless marked "host".  The caller owns
 *    them; the library never frees or retains them after the call returns.
 *  - Coefficients are stored [sample][robot][axis][coeff], C order, contiguous.  In
 *    a batch, problem p's samples follow problem p-1's, so problem p starts at
 *    element sum_{q<p} count_q * n_q * D_q * m_q (m = degree + 1).
 *  - Boundary values are [robot][axis][6] = (p0, v0, a0, pH, vH, aH) per problem,
 *    packed in problem order (eq. boundary_con; both ends give position, velocity
 *    and acceleration).
 *  - Per-sample outputs are packed in sample order across problems.
 *  - Precision SF_FP64: every floating-point array is double.  Otherwise every
 *    floating-point array is float (SF_BF16 / SF_FP16 name the precision of the
 *    fixed-matrix products inside the solver, not of the buffers).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = default stream).
 *  - Errors are returned as sf_status codes; nothing throws across the ABI.  The
 *    message of the last error on the calling thread is sf_last_error().  On any
 *    error nothing has been enqueued.
 */
#ifndef SWARMSF_H
#define SWARMSF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sf_handle_s* sf_handle;

typedef enum {
  SF_OK = 0,
  SF_EINVAL = 1,        /* bad argument: null pointer, size, shape, alignment */
  SF_ENOMEM = 2,        /* device or host allocation failed */
  SF_EDEVICE = 3,       /* a HIP runtime call failed */
  SF_EUNSUPPORTED = 4   /* valid but outside what the kernels implement */
} sf_status;

typedef enum {
  SF_FP64 = 0,          /* everything in double precision */
  SF_FP32 = 1,          /* everything in single precision */
  SF_BF16 = 2,          /* basis products in bf16 MFMA with the rounding residuals of both factors
                           fed back as fp32-accumulated correction terms; fp32 state */
  SF_FP16 = 3           /* the same with fp16.  SF_BF16 / SF_FP16 apply to the problems the MFMA
                           kernels cover (3D, n_robots <= 32, degree <= 15, horizon <= 256); the
                           other problems of the batch run in FP32 (see sf_project).  With
                           SF_RESID_HISTORY or SF_GENERIC_KERNEL they are SF_EUNSUPPORTED */
} sf_precision;

/* Flags for sf_project. */
#define SF_RESID_HISTORY 1   /* resid_out holds every iteration: [S][iters][2] */
#define SF_GENERIC_KERNEL 2  /* use the generic LDS kernel even where the MFMA kernel applies */
#define SF_USE_GRAPH 4       /* capture the launch sequence in a hipGraph on first use (per plan and
                                argument set) and replay it; the first call must not be under capture */
#define SF_AUTOTUNE 8        /* on the first call for a batch and precision (synchronizes): time the
                                MFMA launch candidates (2, 3 or 4 waves per sample; for persistent launches
                                also 1-6 workgroups per CU) on 50 (persistent: 30) iterations of this batch and keep the
                                fastest, also in the JSON-lines cache $SWARMSF_TUNE_CACHE (default
                                ~/.cache/swarmsf_tune.jsonl) for later processes */
#define SF_FP_RESIDUAL 32    /* resid_out is [S][3]: the two residual figures, then the fixed-point
                                residual sum over the iterations, sum_k ||xi^{k+1} - xi^k||^2 +
                                ||lambda^{k+1} - lambda^k||^2 (the first term of eq. NN_loss); not
                                with SF_RESID_HISTORY */
#define SF_PERSISTENT 16     /* run a single-shape batch through the persistent work-queue kernel (a
                                batch of mixed swarm sizes always uses it on the MFMA path) */

/* Per-sample status bits written by sf_project into status_out (0 = finite and converged).
 *  SF_SAMPLE_NONFINITE_INPUT  a coefficient of the sample's xi_bar, xi0 or lam0, or a boundary value of
 *                             its problem, is NaN or infinite.  The sample is not iterated: its xi_out,
 *                             lam_out and resid_out entries are NaN.  Other samples are unaffected.
 *  SF_SAMPLE_NONFINITE        from finite inputs, the iteration produced a NaN or infinity (overflow);
 *                             it stays in the state, so it shows in xi_out / lam_out / resid_out
 *  SF_SAMPLE_NOT_CONVERGED    the largest Euclidean norm of one constraint's block of the final primal
 *                             residual (eq. primal_residual) exceeds SF_CONV_TOL (iters >= 1 only; an
 *                             infeasible problem keeps this bit however long it runs).
 * The finiteness tests are bit tests on the IEEE encoding, so they hold in every kernel. */
#define SF_SAMPLE_NONFINITE_INPUT 1
#define SF_SAMPLE_NONFINITE 2
#define SF_SAMPLE_NOT_CONVERGED 4
#define SF_CONV_TOL 1e-3     /* m, m/s, m/s^2: the feasibility tolerance behind the converged count */

/* One problem shape (eqs. poly, inter_robot_con, workspace_con; the velocity and acceleration
 * bounds are origin-centred balls in the polar form of eq. workspace_polar with d in [0, 1]).
 *  n_robots >= 2, dims in {2, 3}, degree >= 5 (Bernstein), horizon >= degree + 1,
 *  grid tau_h = h / (horizon - 1), h = 0..horizon-1, over [0, t_final] seconds.
 *  safety_a, safety_b: semi-axes of the centre-to-centre spheroid M_a = diag(a, a, b)
 *  (for spheres of radius r, a = b = 2r).  vmax, amax <= 0 switch that bound off.
 *  rho_*: penalty weights of eq. aug_lag per constraint block (the paper uses one
 *  rho; 1.0 for each block reproduces it).
 *  ws_a, ws_b, ws_x, ws_y, ws_z: the workspace spheroid M_w = diag(a_w, a_w, b_w) about the
 *  centre p_w of eq. workspace_con (rows F_w of eq. f_e), in the polar form of eq.
 *  workspace_polar with d in [0, 1]; ws_a <= 0 switches it off (then ws_b, rho_ws and the
 *  centre are ignored).  In 2D only ws_a, ws_x and ws_y count. */
typedef struct {
  int32_t n_robots, dims, degree, horizon;
  double t_final;
  double safety_a, safety_b;
  double vmax, amax;
  double rho_coll, rho_vel, rho_acc;
  double ws_a, ws_b, rho_ws;
  double ws_x, ws_y, ws_z;
} sf_config;

/* A batch of problems (host arrays of length n_problems).  cfg_slot indexes the
 * configs given to sf_setup; sample_count >= 1 is the number of samples. */
typedef struct {
  int32_t n_problems;
  const int32_t* cfg_slot;       /* host */
  const int32_t* sample_count;   /* host */
} sf_batch;

/* Factorise the QP step of eq. (xi_step) for each config, in FP64 on the host, and
 * upload the factors.  The KKT matrix does not depend on the samples (Appendix,
 * "pre-stored factorisations"), so this runs once per shape.  Device memory owned by
 * the handle is released by sf_destroy.  Selects the current HIP device. */
sf_status sf_setup(const sf_config* cfgs, int32_t n_cfgs, sf_handle* out);

void sf_destroy(sf_handle h);

/* Run `iters` fixed-point iterations (eqs. alpha_step .. xi_step) on every sample.
 *  xi_bar  [S, n, D, m]  sampled coefficients (the SF target)
 *  bvals   [P, n, D, 6]  boundary values per problem
 *  xi0     [S, n, D, m]  initial coefficients, or NULL for xi0 = xi_bar
 *  lam0    [S, n, D, m]  initial multipliers, or NULL for zero
 *  iters   >= 0
 *  xi_out  [S, n, D, m]  result (may alias neither input)
 *  lam_out [S, n, D, m]  final multipliers, or NULL
 *  resid_out [S, 2] (or [S, iters, 2] with SF_RESID_HISTORY), or NULL:
 *          (||r_p||_2^2, largest Euclidean norm of one constraint's residual block)
 *          for the primal residual of eq. (primal_residual) after the last step.
 *  status_out int32 [S], or NULL: per-sample SF_SAMPLE_* bits (non-finite input, non-finite result,
 *          not converged), so that non-convergence and NaN are reported as data, not as errors.
 *          Asking for it costs one residual pass per sample when resid_out is NULL.
 *  ckpt    [ceil(iters/ckpt_every), 2, total coefficient elements] or NULL: the state
 *          (xi^k, lambda^k) at k = 0, c, 2c, ... (c = ckpt_every >= 1), as needed by
 *          sf_project_backward.
 * Aliasing: outputs must not overlap inputs or each other.
 * Kernel choice is per problem: with SF_FP32, SF_BF16 or SF_FP16 the problems of a shape the MFMA
 * kernels cover (see SF_FP16) that fits their LDS plan run on them, and the other problems of the
 * batch on the generic kernel in FP32, in a second launch on the same stream (results of every
 * problem as in a batch of its own kind).  SF_FP64, SF_RESID_HISTORY and SF_GENERIC_KERNEL put the
 * whole batch on the generic kernel. */
sf_status sf_project(sf_handle h, const sf_batch* batch, int32_t precision,
                     const void* xi_bar, const void* bvals,
                     const void* xi0, const void* lam0, int32_t iters,
                     void* xi_out, void* lam_out, void* resid_out, int32_t* status_out, int32_t flags,
                     void* ckpt, int32_t ckpt_every, void* stream);

/* Reverse-mode derivative of sf_project (same batch, precision, iters, xi_bar, bvals
 * and the ckpt it wrote) through the unrolled iterations, eq. (NN_loss) style
 * training of the initialisation.  Given cotangents of xi_out, lam_out, of
 * resid_out[:, 0] (g_resid, [S]) and of the fixed-point residual sum of SF_FP_RESIDUAL
 * (w_fpr, [S]) -- each may be NULL = zero -- it writes the gradients with respect to
 * xi0, lam0 and xi_bar (each may be NULL = not wanted).  The workspace rows of eq. (f_e) are
 * differentiated like the bound balls (their projection's 3x3 Jacobian).  The MFMA reverse sweep
 * serves batches whose every problem the MFMA kernels cover (up to 16 robots, no workspace); any
 * other batch runs the generic reverse sweep, which recomputes each checkpoint segment with the
 * generic FP32 (or FP64) iteration. */
sf_status sf_project_backward(sf_handle h, const sf_batch* batch, int32_t precision,
                              const void* xi_bar, const void* bvals, int32_t iters,
                              const void* ckpt, int32_t ckpt_every,
                              const void* g_xi_out, const void* g_lam_out, const void* g_resid,
                              const void* w_fpr, void* g_xi0, void* g_lam0, void* g_xi_bar, void* stream);

/* Constraint violations of coefficient arrays, computed in FP64 on the device at the
 * grid times.  xi is [S, n, D, m] (double for SF_FP64, else float); viol_out is
 * double [S, 5] = (a * (1 - min ||M_a^{-1}(p_i - p_j)||), max ||v|| - vmax,
 * max ||acc|| - amax, max |A xi - b|, a_w * (max ||M_w^{-1}(p_i - p_w)|| - 1), the last 0
 * without a workspace); positive means violated. */
sf_status sf_feasibility(sf_handle h, const sf_batch* batch, int32_t precision,
                         const void* xi, const void* bvals, void* viol_out, void* stream);

/* Equality-only QP layer of the decoders (Sec. IV: the QP of eq. sf_form without its inequality
 * rows, solved in closed form):
 *   xi_out = argmin 1/2 ||xi - xi_in||^2  subject to the boundary rows A xi = b of eq. boundary_con.
 * Those rows involve only the three first and three last coefficients of each robot-axis (the
 * Bernstein end conditions), so the other coefficients pass through and those six become Bmap b
 * (the inverse end-condition block sf_setup stores, see sf_factor_table).
 *  xi_in   [S, n, D, m]  device; double for SF_FP64, float for any other precision
 *  bvals   [P, n, D, 6]  device, boundary values per problem, as for sf_project
 *  xi_out  [S, n, D, m]  device; may be xi_in itself (in place), must not overlap it otherwise
 * The workspace, bounds and penalty weights of the configs play no part.  Errors: SF_EINVAL for
 * NULL or misaligned arrays and bad batches; launch failures as for sf_project. */
sf_status sf_qp_equality(sf_handle h, const sf_batch* batch, int32_t precision, const void* xi_in,
                         const void* bvals, void* xi_out, void* stream);

/* Reverse mode of sf_qp_equality for cotangents g_out [S, n, D, m] of xi_out:
 *  g_xi_in [S, n, D, m]  g_out with the six end coefficients of every robot-axis zeroed, or NULL
 *                        (may be g_out itself)
 *  g_bvals [P, n, D, 6]  per problem, the sum over its samples of Bmap^T g_out[end coefficients],
 *                        summed in a fixed order (deterministic), or NULL
 * Calls on one handle must not overlap in time on different streams: the per-sample-chunk
 * partial sums of g_bvals live in a scratch buffer the handle owns (grown on demand). */
sf_status sf_qp_equality_backward(sf_handle h, const sf_batch* batch, int32_t precision, const void* g_out,
                                  void* g_xi_in, void* g_bvals, void* stream);

/* Allocation-free variant of sf_qp_equality_backward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results, bit for bit.  Instead of the handle's plan tables and its partial-sum buffer
 * (both allocated on first use), it builds the batch's problem and chunk tables with a kernel and keeps
 * them and the per-chunk partial sums in a fixed 16 MiB device array of the library (one per GPU,
 * located at sf_setup, held until the process ends).  It calls no allocating routine.
 *  Limits: at most 64 problems per call, and tables plus partial sums within the 16 MiB (about
 *  (n_chunks x largest n D 6) elements, chunks of max(1, 32768 / (n D m)) samples per problem;
 *  roughly 900K samples of 16 robots in FP32); beyond them SF_EUNSUPPORTED, before anything is
 *  enqueued.
 *  Every call on one GPU shares that array, which keeps the last call's contents: calls that overlap
 *  in time on one GPU (any handle, any stream) race.  Nothing in it needs clearing: each call writes
 *  every entry it reads. */
sf_status sf_qp_equality_backward_noalloc(sf_handle h, const sf_batch* batch, int32_t precision, const void* g_out,
                                          void* g_xi_in, void* g_bvals, void* stream);

/* Host-only inspection of the FP64 factor table sf_setup builds for one config (needs no
 * GPU).  Writes a 16-double header (m, m_f, H, n, then element offsets of basis, X1, X01,
 * Bmap, Gfx, Rfx into the table that follows) and the table; *needed receives the
 * number of doubles required (call with out = NULL to query).  Tables:
 *   basis [3][H][m]  Bernstein position/velocity/acceleration rows at tau_h = h/(H-1)
 *   X1  [m_f][m_f]   (I + n rho_c Gff + Rff)^-1,  X01 = (I + Rff)^-1 - X1, where
 *                    G = P^T P, Rm = rho_v Pd^T Pd + rho_a Pdd^T Pdd, f = free coefficients
 *                    3..degree-3: the free-coefficient block of the inverse KKT matrix of
 *                    eq. (xi_step) is J (x) (X1 + X01) + (I - J) (x) X1 per axis, J = 11^T/n
 *   Bmap [6][6]      pinned coefficients (c0, c1, c2, c_{N-2}, c_{N-1}, c_N) from b
 *   Gfx, Rfx [m_f][6] free x pinned blocks of G and Rm. */
sf_status sf_factor_table(const sf_config* cfg, double* out, int64_t capacity, int64_t* needed);

/* Message of the last error returned on this thread ("" if none). */
const char* sf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SWARMSF_H */
