/*
 * mdpnop.h -- C ABI of the MI355X (gfx950) S_N source-iteration library with
 * an equation-recast neural-operator warm start (arXiv 2509.01416).
 *
 * General conventions
 *   - Field pointers are DEVICE pointers owned by the caller: FP32, cell-major
 *     with x fastest, nx*ny elements.  Quadrature arrays are HOST pointers.
 *   - All work is enqueued on the context's HIP stream.  Every call returns
 *     after its results and statistics are final (a stream synchronisation).
 *   - The context owns its workspaces (allocated on first use, grown when a
 *     larger problem arrives, reused otherwise).  A context is not
 *     thread-safe; use one per host thread.
 *   - No C++ exception crosses this interface.  On error a negative status is
 *     returned and tr_last_error() describes it.
 *   - Quadrature weights must sum to 1 (to 1e-12) and the set must be closed
 *     under mu -> -mu (and eta -> -eta in 2-D).  With this normalisation the
 *     emission density per unit weight is Q = sigma_s*phi + S and
 *     phi = sum_m w_m psi_m, the scalar flux of section 5.1 (Eq. 12, 17); the
 *     paper's weights sum to 2 with a factor 1/2 on the emission, which gives
 *     the same phi.
 */
#ifndef MDPNOP_H
#define MDPNOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TR_OK = 0,
    TR_NOT_CONVERGED = 1,     /* max_iter reached; last iterate returned      */
    TR_RECAST_DIVERGED = 2,   /* recast loop diverged; guess zeroed           */
    TR_ERR_INVALID_ARG = -1,
    TR_ERR_HIP = -2,
    TR_ERR_OOM = -3,
    TR_ERR_NONFINITE = -4
} tr_status;

typedef enum { TR_BC_VACUUM = 0, TR_BC_REFLECTIVE = 1 } tr_bc;

typedef struct tr_context tr_context;
typedef struct no_model no_model;

/* One fixed-source problem: section 5.1 Eq. 12 (dim = 1) or its x-y analogue
 * (dim = 2).  The parameter vector p of Eq. 1 is (sigma_t, sigma_s).
 * Uniform cells: dx = lx/nx, dy = ly/ny (ny = 1, ly ignored when dim = 1).
 * Requirements: sigma_t > 0, 0 <= sigma_s <= sigma_t, all values finite;
 * sigma_a = sigma_t - sigma_s must not vanish everywhere unless some face is
 * vacuum.  bc = {x-, x+, y-, y+} (tr_bc); only bc[0..1] are used in 1-D.
 * sigma_s1: first Legendre moment of the scattering cross section (linearly
 * anisotropic scattering, section 5.1 Eq. 25), a DEVICE field like
 * sigma_s with |sigma_s1| <= sigma_s, or NULL for isotropic scattering.  The
 * emission of direction Omega_m is then
 *     sigma_s phi + 3 sigma_s1 Omega_m . J + S,  J = sum_m w_m Omega_m psi_m,
 * with J of the previous sweep (the paper's 1/2 and 3/2 factors belong to
 * its weights summing to 2).  Read by tr_solve / tr_solve_noalloc (a 2-D
 * solve with it runs the generic sweep, one direction per lane); not by
 * tr_sweep (a bare sweep has no current) nor by no_recast_guess (the
 * network sees only the isotropic problem, Eq. 23); the eigenvalue solvers
 * reject it.                                                              */
typedef struct {
    int32_t dim, nx, ny;
    double lx, ly;
    const float *sigma_t, *sigma_s, *source;
    int32_t bc[4];
    const float *sigma_s1;
} tr_problem;

/* Discrete ordinates (section 5.1: S_N angular discretisation).  HOST
 * arrays of n_dir entries; eta = NULL in 1-D.  sum(w) = 1.                 */
typedef struct {
    int32_t n_dir;
    const double *mu, *eta, *w;
} tr_quadrature;

/* Per-instance results.  residual: last relative change norm (FP64);
 * balance_rel: |sum q V - sum sigma_a phi V - leakage| / sum q V in FP64;
 * seconds: wall time of the whole call (same value for every instance).   */
typedef struct {
    int32_t status, iterations;
    double residual, balance_rel, seconds;
} tr_stats;

/* Create a context bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *ctx is set on success.        */
tr_status tr_context_create(tr_context **ctx, void *hip_stream);
void tr_context_destroy(tr_context *ctx);
/* Message of the last failed call on ctx ("" if none); valid until the next
 * call on ctx.                                                              */
const char *tr_last_error(const tr_context *ctx);

/*
 * One transport sweep for each of n_inst problems (the operator Sweep of the
 * source iteration, section 5.1 after Eq. 20): given the emission density
 * emission[i] (= sigma_s*phi + S per unit weight), solve every direction in
 * upwind order with diamond differencing and return
 * phi_out[i] = sum_m w_m psi_m at cell centres.  sigma_s and source of the
 * problems are not read.  Reflective faces receive zero incoming flux (there
 * is no previous sweep); vacuum faces zero as always.
 * Returns TR_OK or an error.  A 2-D grid too wide for the sweep's on-chip
 * face ring (about 38,000 cells in x at 160 KB of LDS per workgroup) is
 * rejected with TR_ERR_INVALID_ARG before anything is launched; the same
 * holds for tr_solve.                                                       */
tr_status tr_sweep(tr_context *ctx, int32_t n_inst, const tr_problem *p,
                   const tr_quadrature *q, const float *const *emission,
                   float *const *phi_out);

/*
 * Source iteration (the model-based operator M of Eq. 3a/4b; Eq. 9a/10b
 * when phi_init is a neural-operator guess): repeat
 *     phi <- Sweep(sigma_s*phi + S)
 * until the FP64 change norm drops below tol, for n_inst independent
 * problems of possibly different sizes in one batched launch sequence.
 *   tol > 0: relative L2 change ||phi_new - phi_old|| / ||phi_new||;
 *   tol < 0: max_i |phi_new - phi_old| / |phi_new| < -tol.
 * phi_init == NULL or phi_init[i] == NULL -> zero start for instance i;
 * otherwise phi_init[i] (device, may equal phi_out[i]) is the first iterate
 * and reflective faces start isotropic at the adjacent cell's value.
 * Reflective faces are lagged one iteration.  phi_out[i] receives the last
 * iterate; stats[i] (may be NULL) the per-instance results.  Return value:
 * the worst status over instances (errors < 0 take precedence).            */
tr_status tr_solve(tr_context *ctx, int32_t n_inst, const tr_problem *p,
                   const tr_quadrature *q, const float *const *phi_init,
                   float *const *phi_out, double tol, int32_t max_iter,
                   tr_stats *stats);

/*
 * tr_solve without any allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Arguments, results, kernels and launch shapes are those of
 * tr_solve (same answers bit for bit).  Every device workspace of the call
 * lives in one fixed device array of 128 MiB compiled into the library, of
 * which each device holds its own copy until the process ends; the host
 * staging area (2 MiB) is allocated with the context.  The call allocates
 * nothing, on the device or the host; a problem set whose workspace (about
 * 4 * (4 * S + 2) * cells bytes per problem plus its boundary faces and
 * tables; about 90 MB for 16 problems of 256 x 256 at S16) exceeds the array, or
 * whose tables exceed the staging area, is rejected with
 * TR_ERR_INVALID_ARG before anything is launched.  All calls on one device
 * share the array (it keeps the last call's contents; the call initialises
 * everything it reads): calls that overlap on one device, from any context
 * or thread, race.  Kernel timing (tr_profile_enable) is not recorded.     */
tr_status tr_solve_noalloc(tr_context *ctx, int32_t n_inst, const tr_problem *p,
                           const tr_quadrature *q, const float *const *phi_init,
                           float *const *phi_out, double tol, int32_t max_iter,
                           tr_stats *stats);

/* Stopping rule of tr_solve on a context.  The paper quotes only a
 * tolerance for its iterations (section 5.1); these are the two readings.
 *   TR_STOP_CHANGE (default): the change norm of tr_solve's tol (relative L2
 *     for tol > 0, max relative for tol < 0) drops below |tol|.
 *   TR_STOP_ERROR_BOUND: with r_l the relative L2 change of iteration l and
 *     rho = r_l / r_(l-1) the observed contraction rate of the fixed-point
 *     iteration, stop once rho < 1 and r_l rho / (1 - rho) < tol, an
 *     estimate of the remaining distance to the fixed point (for slowly
 *     converging problems, where a small change still leaves a large error).
 *     Needs tol > 0 (else TR_ERR_INVALID_ARG from tr_solve).  stats.residual
 *     still reports r_l.
 * The setting stays on the context until changed; the eigenvalue solvers'
 * inner iterations always use TR_STOP_CHANGE.  Unknown values give
 * TR_ERR_INVALID_ARG.                                                      */
typedef enum { TR_STOP_CHANGE = 0, TR_STOP_ERROR_BOUND = 1 } tr_stop_rule;
tr_status tr_set_stop_rule(tr_context *ctx, int32_t rule);

/* Per-instance results of tr_eigen.  outer: outer updates performed;
 * inner: source-iteration sweeps summed over all inner solves; k: final
 * eigenvalue; dk, dphi: the last update's |k_new - k|/k_new and
 * max|phi_new - phi|/max|phi_new|; balance_rel: particle balance of the last
 * inner solve (fission emission against absorption plus leakage, FP64).   */
typedef struct {
    int32_t status, outer, inner;
    double k, dk, dphi, balance_rel, seconds;
} tr_eigen_stats;

/*
 * One-group k-eigenvalue (section 5.2, Eq. 26; Appendix A2, Eq. A1-A4):
 * the fixed source of each problem is replaced by the fission emission
 * nu_sigma_f*phi/k (per unit weight), and power iteration solves
 *   inner M:  source iteration of the fixed-source problem with source
 *             S = nu_sigma_f*phi/k, warm-started from phi, to tol_inner
 *             (same norm convention as tr_solve's tol) or max_inner sweeps;
 *   outer P:  F(phi) = sum nu_sigma_f*phi*V (FP64),
 *             k <- k*F(phi_half)/F(phi),  phi <- phi_half/F(phi_half),
 * until |dk|/k < tol_k and max|dphi|/max|phi| < tol_phi, or max_outer
 * updates.  nu_sigma_f[i]: DEVICE field (cells, >= 0, finite); the
 * problems' source pointers are not read (may be NULL).  phi_init[i]
 * (device, may equal phi_out[i]; NULL array or entry = flat start) must give
 * F > 0; k_init (HOST, n_inst values > 0; NULL = 1.0) is the starting
 * eigenvalue.  On return phi_out[i] is the eigenfunction normalised to
 * F(phi) = 1 and stats[i] (may be NULL) holds k and the counters.  All
 * instances run as one batch; each stops on its own test.  Status per
 * instance: TR_OK, TR_NOT_CONVERGED (max_outer reached) or
 * TR_ERR_NONFINITE; invalid data (negative or non-finite nu_sigma_f, a start
 * without fissions, the tr_solve field checks) gives TR_ERR_INVALID_ARG
 * before any iteration.  The context keeps a workspace of two fields per
 * instance between calls.                                                  */
tr_status tr_eigen(tr_context *ctx, int32_t n_inst, const tr_problem *p,
                   const float *const *nu_sigma_f, const tr_quadrature *q,
                   const float *const *phi_init, float *const *phi_out,
                   const double *k_init, double tol_k, double tol_phi,
                   double tol_inner, int32_t max_outer, int32_t max_inner,
                   tr_eigen_stats *stats);

/*
 * Equation-recast guess (Eq. 24; Eq. 8 in general form): with the network
 * m trained at (sigma_t_star, sigma_s_star), iterate
 *     phi^(k+1) = NO[ S + (sigma_a* - sigma_a) phi^(k) ],  phi^(0) = 0,
 * where NO(S) = s * net(S/s, x, y) / sigma_a*, s = mean|S| per instance,
 * until ||phi^(k+1)-phi^(k)||/||phi^(k+1)|| < tol or max_iter updates.
 * Problems must be 2-D.  A problem whose grid differs from the network's
 * (a multiple of it) is block-averaged onto the network grid for the loop
 * and the result is bilinearly interpolated back (cell-centred, edges
 * clamped).  An instance also stops (status TR_OK) when it has stalled
 * close to the tolerance: the relative change is below 10 tol but no lower
 * than 0.9 times its value three updates earlier (the network's rounding
 * floor).  On divergence (non-finite change, or an absolute change that
 * grew three times running past the first update's) phi_guess[i] is zeroed
 * and status TR_RECAST_DIVERGED reported, so that a following tr_solve
 * falls back to the zero start.  Per-instance stats: status (TR_OK,
 * TR_NOT_CONVERGED or TR_RECAST_DIVERGED), iterations = network
 * evaluations, residual = last relative change; balance_rel is NaN (no
 * transport balance is defined for the network iterate).  Requirements:
 * 2-D problems on a square grid that is a multiple of the network grid,
 * sigma_t* > sigma_s* >= 0, tol >= 0, max_iter >= 1.                     */
tr_status no_recast_guess(tr_context *ctx, const no_model *m, int32_t n_inst,
                          const tr_problem *p, double sigma_t_star,
                          double sigma_s_star, double tol, int32_t max_iter,
                          float *const *phi_guess, tr_stats *stats);

/* Multigroup data of one problem (section 5.3, Eq. 27-29; Tables 8-9).
 * DEVICE fields (cells, as tr_problem's): sigma_t[g], nu_sigma_f[g] for
 * g < n_groups; sigma_s[g*n_groups + h] is the g -> h scattering field,
 * NULL meaning zero; the within-group field g -> g is required; upscatter
 * (h < g) must be NULL.  chi: HOST array of n_groups fission-spectrum
 * fractions (>= 0, not all zero).  n_groups <= 8.                         */
typedef struct {
    int32_t n_groups;
    const float *const *sigma_t;
    const float *const *sigma_s;
    const float *const *nu_sigma_f;
    const double *chi;
} tr_multigroup;

/*
 * Multigroup k-eigenvalue with downscatter (section 5.3, Eq. 27-29; the
 * power iteration of Appendix A2).  Per outer iteration the groups are
 * solved in order (Gauss-Seidel in energy; exact for the fixed fission
 * source without upscatter), group g by source iteration to tol_inner on
 *   chi_g * sum_h nu_sigma_f_h phi_h / k  (previous outer iterate)
 *   + sum_{h<g} sigma_s^{h->g} phi_h      (this pass's solutions),
 * warm-started from the current iterate; then k <- k F(phi_half)/F(phi) and
 * phi <- phi_half / F(phi_half) with F(phi) = sum_g sum nu_sigma_f_g phi_g V,
 * stopping as tr_eigen with the change norm over all groups.
 * geom[i]: grid, extents and faces of problem i (its field pointers are
 * not read); mg[i]: its data (the same n_groups for every problem).
 * phi_init / phi_out: n_inst*n_groups DEVICE fields, entry i*n_groups + g
 * (phi_init NULL = flat start).  k_init, tolerances, stats as in tr_eigen;
 * stats[i].inner sums the sweeps of all groups; balance_rel sums the group
 * balances (sources against removal and leakage).                         */
tr_status tr_eigen_mg(tr_context *ctx, int32_t n_inst, const tr_problem *geom,
                      const tr_multigroup *mg, const tr_quadrature *q,
                      const float *const *phi_init, float *const *phi_out,
                      const double *k_init, double tol_k, double tol_phi,
                      double tol_inner, int32_t max_outer, int32_t max_inner,
                      tr_eigen_stats *stats);

/* Neural-operator variants of the eigenvalue loop (Appendix A2).          */
typedef enum { NO_EIGEN_SP = 0, NO_EIGEN_CP = 1 } no_eigen_variant;

/*
 * Neural-operator outer loop of the one-group k-eigenvalue problem
 * (section 5.2; Appendix A2 (i) simple preconditioning, Eq. A5, and (ii)
 * constrained preconditioning, Eq. A7-A8).  Per outer update:
 *   u = NO[ S + (sigma_a* - sigma_a) phi ],  S = nu_sigma_f*phi/k,
 * with NO as in no_recast_guess (one network application); NO_EIGEN_CP
 * then applies one transport sweep of sigma_s*u + nu_sigma_f*u/k; then the
 * outer update of tr_eigen (k, normalisation F(phi) = 1, the same stopping
 * test on tol_k and tol_phi).  The result is the starting pair for the
 * model-based refinement of Eq. A6: call tr_eigen with phi_init = phi_out
 * and k_init = stats[i].k.  Problems: 2-D on the network's 64 x 64 grid,
 * vacuum faces; the source fields are not read.  Arguments as in tr_eigen;
 * q is used by NO_EIGEN_CP's sweep (and checked for both).  stats[i].inner
 * counts transport sweeps (0 for SP); balance_rel is NaN.  Batch limit as
 * in no_recast_guess.                                                      */
tr_status no_eigen(tr_context *ctx, const no_model *m, int32_t n_inst,
                   const tr_problem *p, const float *const *nu_sigma_f,
                   const tr_quadrature *q, double sigma_t_star, double sigma_s_star,
                   int32_t variant, const float *const *phi_init,
                   float *const *phi_out, const double *k_init, double tol_k,
                   double tol_phi, int32_t max_outer, tr_eigen_stats *stats);

/* ---------------------------------------------------------------------
 * Fourier neural operator (section 4.2, Appendix A1; 2-D form): lift of
 * (field, x, y) to `width` channels, `layers` Fourier layers (retained
 * modes kx in [0,modes), ky in [0,modes) U [grid-modes, grid)), GELU after
 * all but the last, projection width -> 128 -> 1.  Supported shape:
 * width 32, modes 12, layers 4, grid 64.  Parameters are a flat FP32
 * vector (master copy) in this order:
 *   W0[3][w], b0[w]; per layer R[2][m][m][w][w][2], W[w][w], b[w];
 *   P1[w][128], c1[128], P2[128], c2[1]
 * (2,368,001 values for the supported shape).  The network computes on
 * the matrix cores with FP32 accumulation; operands are rounded to BF16
 * when staged (see no_model_set_fp32).  params_host may be NULL (all
 * parameters zero).  The model lives on the context's device.
 * ------------------------------------------------------------------- */
tr_status no_model_create(tr_context *ctx, no_model **m, int32_t width,
                          int32_t modes, int32_t layers, int32_t grid,
                          const float *params_host);
/* Deep operator network (section 4.1, Eq. 11; Appendix A1 carried to the
 * x-y grid): a branch net maps the input field sampled at the grid's
 * grid*grid cells to `basis` coefficients through layers of `hidden`
 * units, a trunk net maps each cell centre (x/lx, y/ly) to `basis` values,
 * and the output at a cell is their inner product.  Both nets are fully
 * connected with ReLU between layers and linear last layers; no bias on
 * the inner product.  Supported shape: grid 64, hidden 200, basis 100 (the
 * paper's hidden sizes; 940,600 parameters).  Parameters (flat FP32, input
 * index first in every weight matrix):
 *   W1[P][h], b1[h], W2[h][h], b2[h], W3[h][k], b3[k],   branch (P = grid^2)
 *   V1[2][h], c1[h], V2[h][h], c2[h], V3[h][k], c3[k]    trunk
 * The model handle is used like the Fourier operator's by no_forward,
 * no_train_step, no_recast_guess, no_eigen and the parameter / state calls;
 * operands are rounded to BF16 on the matrix cores (FP32 with
 * no_model_set_fp32).  The trunk's basis is kept on the device and
 * recomputed when the parameters change.                                  */
tr_status no_model_create_deeponet(tr_context *ctx, no_model **m, int32_t grid,
                                   int32_t hidden, int32_t basis, const float *params_host);
void no_model_destroy(no_model *m);
int64_t no_model_param_count(const no_model *m);
/* Copy the FP32 master parameters to host memory (param_count floats).   */
tr_status no_model_get_params(tr_context *ctx, const no_model *m,
                              float *params_host);
/* Replace the FP32 master parameters from host memory; also clears the
 * Adam moments and step count (a new starting point for training).        */
tr_status no_model_set_params(tr_context *ctx, no_model *m,
                              const float *params_host);
/* Training checkpoint: the FP32 master parameters, Adam's first and second
 * moments (each param_count floats, HOST buffers) and the count of Adam
 * steps taken (its bias corrections depend on it).  Setting a state taken
 * with no_model_get_state and continuing to train reproduces the
 * uninterrupted run bit for bit.  set_state rejects a negative step.      */
tr_status no_model_get_state(tr_context *ctx, const no_model *m, float *params_host,
                             float *adam_m_host, float *adam_v_host, int64_t *step);
tr_status no_model_set_state(tr_context *ctx, no_model *m, const float *params_host,
                             const float *adam_m_host, const float *adam_v_host,
                             int64_t step);
/* Operand precision of the matrix-core products: enable = 0 (default)
 * rounds operands to BF16, enable = 1 keeps them FP32
 * (v_mfma_f32_16x16x4f32; slower, for checking against FP64 references).
 * Accumulation is FP32 either way.                                         */
tr_status no_model_set_fp32(no_model *m, int32_t enable);

/* Network forward for a batch: input[b] and output[b] are device
 * grid*grid FP32 fields (the first input channel; the coordinate channels
 * are generated inside).  1 <= batch <= 65535 (also for no_train_step and
 * n_inst of no_recast_guess), else TR_ERR_INVALID_ARG.                     */
tr_status no_forward(tr_context *ctx, const no_model *m, int32_t batch,
                     const float *input, float *output);

/* One training step on a batch (Appendix A1: Adam, MSE loss): forward,
 * MSE against target, hand-written backward, Adam (b1 0.9, b2 0.999,
 * eps 1e-8, bias-corrected) on the FP32 master parameters, BF16 copy
 * refreshed.  input/target: device [batch][grid*grid].  *loss receives the
 * batch MSE before the update.  grad_out (device, param_count floats, may
 * be NULL) receives the gradient; with lr = 0 the parameters are unchanged
 * and the call only evaluates the loss and gradient.  Returns
 * TR_ERR_NONFINITE (parameters already updated) if the loss is not finite. */
tr_status no_train_step(tr_context *ctx, no_model *m, int32_t batch,
                        const float *input, const float *target, double lr,
                        double *loss, float *grad_out);

/* ---------------------------------------------------------------------
 * Host-only helpers and tuning
 * ------------------------------------------------------------------- */

/* Run the host-side argument checks of tr_solve (problem shapes, extents,
 * boundary codes, quadrature symmetry and normalisation, tol, max_iter)
 * without touching a device; field values are not read.  msg (may be NULL)
 * receives the reason for a failure, truncated to msg_len bytes.          */
tr_status tr_check_args(int32_t n_inst, const tr_problem *p,
                        const tr_quadrature *q, double tol, int32_t max_iter,
                        char *msg, int32_t msg_len);

/* Force the 2-D sweep's launch shape on this context (0 = automatic):
 * D directions per lane (1,2,3,4,6,9), W waves per workgroup (1..16),
 * S direction slices per octant, R rows per lane segment (a power of two
 * <= 64; a problem narrower than R uses the automatic choice).  Every
 * configuration sums partial fluxes in a fixed order, so a given
 * configuration reproduces its result bit for bit; different
 * configurations agree to FP32 rounding.                                  */
tr_status tr_set_sweep_config(tr_context *ctx, int32_t D, int32_t W, int32_t S,
                              int32_t R);

/* Autotuner: times every feasible launch shape (D in 1..4 directions per
 * lane, W waves per workgroup from a fixed set plus, for one direction per
 * lane, every ceil(nd/S) for an octant of nd directions; slices and block
 * size then chosen by the planner) with `reps` HIP-event-timed sweeps of these problems (their
 * sources as emission; one untimed sweep first), each followed by the sum
 * of its partial scalar-flux planes (their number depends on the shape),
 * times the shapes within
 * 5 % of the fastest again in three interleaved rounds, and leaves the one
 * with the lowest total forced on the context exactly as
 * tr_set_sweep_config would (reset with
 * tr_set_sweep_config(ctx, 0, 0, 0, 0)).  out6 (may be NULL) receives the
 * chosen plan as tr_get_sweep_plan reports it, best_ms (may be NULL) its
 * time per sweep and plane sum.  2-D only: for 1-D problems nothing is tuned.  Allocates
 * one temporary output array per call.                                    */
tr_status tr_autotune(tr_context *ctx, int32_t n_inst, const tr_problem *p,
                      const tr_quadrature *q, int32_t reps, int32_t *out6,
                      double *best_ms);

/* Sweep kernel selection on this context: generic = 0 (default) uses the
 * specialised 2-D kernel whenever every problem of a call has only vacuum
 * faces and a grid it takes (64-row lane segments, the last row block
 * possibly ragged: several row blocks with nx >= 63 + KB, or one with
 * nx >= ny - 1; tr_get_sweep_plan reports the choice), the generic kernel
 * otherwise;
 * generic = 1 always uses the generic kernel.  Both perform the same
 * floating-point operations in the same order, so for one launch shape
 * their results agree bit for bit.                                        */
tr_status tr_set_sweep_kernel(tr_context *ctx, int32_t generic);

/* Persistent iteration (enable = 1; off by default): when a 2-D solve runs
 * the specialised sweep with one direction per lane (any wave count), and
 * every workgroup of the launch can be resident at once,
 * tr_solve and the eigenvalue solvers run each chunk of source iterations
 * (the batched-launch pattern of the sweeps of section 5.1) as one
 * cooperative launch: per iteration the workgroups of each instance sweep,
 * meet at a barrier in device memory, combine their share of the
 * instance's cells, meet again and evaluate the convergence test.  Results,
 * iteration counts and statuses equal those of the per-kernel launches
 * (enable = 0) bit for bit.  spin_limit > 0 bounds the polls of a barrier
 * wait (0 selects the default, 2^18 polls, far above a normal wait); a
 * wait that runs out ends every wait of the launch, whose workgroups all
 * finish, and the call returns TR_ERR_HIP ("barrier wait timed out").
 * Instances never wait on each other.  On gfx950 it is slower than the
 * per-kernel launches (an instance barrier of its workgroups costs more
 * than the kernel boundary it replaces), hence opt-in.                    */
tr_status tr_set_persistent(tr_context *ctx, int32_t enable, int32_t spin_limit);

/* Debugging: with enable = 1 every HIP step of a call on this context
 * (launch, copy) is followed by a stream synchronisation and an error
 * check, so a failing kernel is reported, in tr_last_error, at the step
 * that launched it rather than at the next synchronisation.  Slow; off by
 * default, or on for every new context when the environment variable
 * MDPNOP_SYNC_CHECKS is set to a value other than 0.                      */
tr_status tr_set_sync_checks(tr_context *ctx, int32_t enable);

/* Kernel timing for benchmarks: with enable != 0, tr_solve records HIP
 * events on the context stream around every sweep launch and around every
 * combine+finalize pair (totals reset by each call of this function).    */
tr_status tr_profile_enable(tr_context *ctx, int32_t enable);
/* out4 = {sweep ms, sweep launches, combine+finalize ms, their count}.   */
tr_status tr_profile_read(tr_context *ctx, double *out4);
/* out6 = out4 followed by {persistent-iteration ms, its launches} (each
 * persistent launch runs a chunk of source iterations: sweeps, combines
 * and convergence tests).                                                 */
tr_status tr_profile_read_ex(tr_context *ctx, double *out6);

/* The launch shape the next tr_solve / tr_sweep on these problems would
 * use: out6 = {D, W, S of problem 0, R of problem 0, KB, specialised
 * kernel (1) or generic (0)}.  ctx may be NULL (host-only: default limits,
 * automatic choices); field pointers are not read.                        */
tr_status tr_get_sweep_plan(tr_context *ctx, int32_t n_inst,
                            const tr_problem *p, const tr_quadrature *q,
                            int32_t *out6);

#ifdef __cplusplus
}
#endif

#endif /* MDPNOP_H */
