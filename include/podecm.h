/*
 * podecm.h -- C ABI of the hyper-reduced (POD + ECM + geometrical
 * transformation) microscale solve of Guo, Rokos & Veroy, arXiv 2307.16894.
 *
 * The library solves, for a batch of independent macroscopic points, the
 * reduced RVE problem of Sec. 3.2 (eqs. forcevector_ecm and
 * stiffnessmatrix_ecm) by Newton's method on the reduced coordinates
 * (eq. red_newton), with the finite-strain J2 model of Appendix A at the ECM
 * points, and returns the effective stress and stiffness of Sec. 3.3
 * (eqs. eff_stress_1, tangent_problem_red, eff_stiffness_1).  The calls
 * follow the paper's statement of the two-scale problem (Fig. 1 and
 * Algorithm 1, online part): given Fbar and mu, with history, return Pbar
 * and Abar.
 *
 * Conventions
 * -----------
 * - Every per-call and state buffer is device memory owned by the caller
 *   (plain pointers).  The library owns only the ROM constants uploaded by
 *   rom_load.  Nothing in rom_step allocates.
 * - All device work is enqueued on the caller's stream and is asynchronous;
 *   the only host synchronisation is inside rom_load (upload) and
 *   rom_state_init (to report invalid shape parameters).
 * - 2x2 tensors are stored row-major as [11, 12, 21, 22]; 4x4 tangents
 *   A[(ij)(kl)] = dP_ij / dF_kl row-major over those index pairs.
 * - Return value: ROM_OK or a negative ROM_E* code.  Per-point Newton
 *   failures are not call errors; they are reported in status[].
 */
#ifndef PODECM_H
#define PODECM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define ROM_OK           0
#define ROM_EINVAL      -1  /* bad argument (null pointer, size out of range) */
#define ROM_EFORMAT     -2  /* artifact malformed (magic, sizes, non-finite data, w_q <= 0) */
#define ROM_EVERSION    -3  /* artifact version not supported */
#define ROM_EHIP        -4  /* a HIP runtime call failed */
#define ROM_EINVAL_MU   -5  /* some shape parameters give det F_mu <= 0 at an ECM point */
#define ROM_EUNSUPPORTED -6 /* option combination not built */
#define ROM_ESCRATCH    -7  /* rom_step_noalloc: the batch exceeds its static scratch (ROM_NOALLOC_MAX_BATCH) */

/* per-point status written by rom_step */
#define ROM_ST_CONVERGED 0  /* ||f||_2 <= tol at the returned state */
#define ROM_ST_MAXITER   1  /* iteration cap reached; nothing committed */
#define ROM_ST_NONFINITE 2  /* non-finite residual; nothing committed */
#define ROM_ST_FALLBACK  3  /* converged after the learned warm start fell back to the plain guess */
#define ROM_ST_BADMU     4  /* the point's shape parameters were rejected */

/* contraction precision of the reduced tangent K (Sec. 3.2, eq. stiffnessmatrix_ecm) */
#define ROM_DT_F64  0
#define ROM_DT_F32  1
#define ROM_DT_BF16 2

#define ROM_MAX_SUBSTEPS 12  /* largest load-step cutting depth */

/* execution form of rom_step */
#define ROM_MODE_STAGED 0  /* one kernel per stage, host-enqueued Newton loop */
#define ROM_MODE_FUSED  1  /* one persistent kernel, device-side Newton loop */
#define ROM_MODE_PHASED 2  /* the first Newton evaluations of every point as a material launch (one lane per
                              ECM point of every point) and a contraction + elimination launch each, the points
                              still running after them finished by the fused kernel from where they stand
                              (n <= 75); same arithmetic, and bit for bit the same results, as ROM_MODE_FUSED.
                              Eager launches only: inside a stream capture rom_step returns ROM_EUNSUPPORTED */

/* initial guess of the Newton iteration */
#define ROM_WARM_PREV 0  /* the committed r (plain guess) */
#define ROM_WARM_MLP  1  /* committed r + the increment predicted by a warm-start network */

typedef struct rom_model* rom_handle;
typedef struct rom_mlp* rom_mlp_handle;

typedef struct rom_opts {
  double  tol;          /* absolute tolerance on ||f||_2 (default 1e-8) */
  int32_t max_iter;     /* Newton evaluations per step, >= 1 (default 15) */
  int32_t fixed_iters;  /* 1: make exactly max_iter evaluations, status from the last (parity mode) */
  int32_t commit;       /* 1: converged points commit r, history and Fbar */
  int32_t contraction;  /* ROM_DT_*: precision of the K contraction; all else is FP64 */
  int32_t mode;         /* ROM_MODE_* */
  int32_t warm_start;   /* ROM_WARM_*; ROM_WARM_MLP needs mode FUSED or PHASED and mlp */
  int32_t split;        /* fused and phased forms: -1 automatic, 0 the waves of a workgroup split the ECM points,
                           1 they split the column tiles of K (needed for n > 75 in FP64) */
  int32_t grid_per_cu;  /* fused form: 0 one workgroup per point; k > 0 persistent grid of k workgroups per
                           compute unit pulling points from a device-side work list (phased form: the grid of
                           its fused part, 0 meaning 2) */
  int32_t max_substeps; /* fused and phased forms, commit only: load-step cutting depth D (0..ROM_MAX_SUBSTEPS, default 0,
                           the plain step).  A step that fails is retried towards targets
                           Fbar_c + (t / 2^D)(Fbar - Fbar_c) on the segment from the committed Fbar_c, halving the
                           stride on failure and doubling it after a converged sub-step, which is committed at once
                           (the material-model appendix: the global Newton solve may need much smaller load steps).
                           The point fails when a stride of 1 / 2^D fails; its committed state is then the last
                           converged sub-step.  iters counts the evaluations of all attempts. */
  int32_t phased_evals; /* phased form: evaluations made by the phased launches (0: 6, or 4 with the learned
                           warm start, which needs fewer; at most max_iter); the rest of the step runs in the
                           fused kernel, and so does an attempt that fails with load-step cutting on (from its
                           start) */
  int32_t phased_early; /* phased form: after this many evaluations the points whose ||f|| stayed above 0.3 of
                           the previous evaluation's (slow convergence: likely to fail the plain step and be cut
                           into sub-steps) go to a fused kernel on a side stream, beside the remaining phased
                           evaluations (0: 3, or none with the learned warm start; -1: none; used when below
                           phased_evals) */
  int32_t abar_f64;     /* FP32 / BF16 contraction, fused and phased forms: 1 forms Abar (and the K*^-1 C kept for
                           the shape sensitivities) at the converged points from one more evaluation at the
                           returned state with the FP64 contraction, so that K* is the FP64 K there (Sec. 3.3);
                           the final commit of those points follows that evaluation.  0 (default): K*, C and
                           sum w|J| A of the last evaluation, in the contraction precision.  No effect with the
                           FP64 contraction. */
  rom_mlp_handle mlp;   /* network for ROM_WARM_MLP (see below), else NULL */
  const int32_t* active;  /* device i32 [batch] or NULL: points with active[p] == 0 are skipped, their state
                             and outputs untouched (fused and phased forms) */
} rom_opts;

/* Fill *o with the defaults: tol 1e-8, max_iter 15, commit, FP64, staged form, plain guess, split -1,
   no load-step cutting. */
int rom_default_opts(rom_opts* o);

/*
 * rom_load -- parse a ROM artifact (the output of the offline stage of
 * Algorithm 1: ECM weights and points, parent gradients of the POD modes and
 * of the auxiliary transformation modes at those points, material constants,
 * mu -> c map) and upload it to `device`.  The maps from the shape
 * parameters mu to the affine coefficients c of the transformation
 * (Sec. 3.4, the auxiliary problem with affine boundary data): kind 0, one
 * axis-aligned elliptical void, mu = (a, b), c = mu / r0 - 1; kind 1, four
 * rotated voids of fixed area, mu = (kappa_i, theta_i); kind 2, inclusions
 * all scaled about their centres (Sec. 4.1), mu = (zeta), c = zeta - 1.
 *   blob/bytes : host memory holding the artifact file; read only, not retained.
 *   device     : HIP device ordinal; made current during the call.
 *   out        : receives the handle; release with rom_free.
 * Errors: ROM_EINVAL, ROM_EFORMAT (bad magic, truncated, non-finite values,
 * a weight <= 0), ROM_EVERSION, ROM_EHIP.
 */
int rom_load(const void* blob, size_t bytes, int device, rom_handle* out);
int rom_load_file(const char* path, int device, rom_handle* out);
int rom_free(rom_handle h);

/* Sizes of a loaded ROM: modes n, ECM points m, affine coefficients c, shape parameters per point. */
int rom_info(rom_handle h, int32_t* n, int32_t* m, int32_t* c, int32_t* n_mu);

/*
 * State of a batch of macro points, in one caller-allocated device buffer:
 * committed and trial reduced coordinates r, committed and trial history
 * (F^pl in-plane, F^pl_33, xi per ECM point: the appendix's internal
 * variables), the transformation cached at the ECM points, the last
 * effective stress / stiffness, and Newton workspace.  rom_state_bytes gives
 * its size (256-byte aligned fields); rom_state_offsets gives the byte offset
 * of each field (ROM_FIELD_*), for checkpointing and inspection.
 */
#define ROM_FIELD_R_COMMITTED 0  /* f64 [batch][n] */
#define ROM_FIELD_R_TRIAL     1  /* f64 [batch][n] */
#define ROM_FIELD_H_COMMITTED 2  /* f64 [batch][6][m]: Fp11 Fp12 Fp21 Fp22 Fp33 xi, point fastest */
#define ROM_FIELD_H_TRIAL     3  /* f64 [batch][6][m] */
#define ROM_FIELD_TRANSFORM   4  /* f64 [batch][5][m]: F_mu^-1 (4), w_q |det F_mu| */
#define ROM_FIELD_PBAR        5  /* f64 [batch][4]  last effective stress */
#define ROM_FIELD_ABAR        6  /* f64 [batch][16] last effective stiffness */
#define ROM_FIELD_MU_OK       7  /* i32 [batch] 1 if the shape parameters were accepted */
#define ROM_FIELD_FBAR_COMMITTED 8  /* f64 [batch][4] Fbar of the last committed step (I initially) */
#define ROM_FIELD_R_GUESS     9  /* f64 [batch][n] initial guess used by the last rom_step */
#define ROM_FIELD_SUBSTEPS   10  /* u32 [batch] converged (sub-)steps of the last rom_step: bit k is set when one
                                    ended at t = (k+1)/32 of the segment from the committed Fbar to Fbar (exact
                                    up to cutting depth 5; deeper, the 1/32 cell holding the end).  A plain step
                                    that converges sets bit 31 alone; 0 when none converged.  Two runs followed
                                    the same loading path through a step when their records agree (written by
                                    every form; untouched for inactive points) */
#define ROM_NFIELDS           11
int rom_state_bytes(rom_handle h, int32_t batch, size_t* bytes);
int rom_state_offsets(rom_handle h, int32_t batch, size_t* offsets /* [ROM_NFIELDS] */);

/*
 * rom_state_init -- Algorithm 1 online, step 1: for each point evaluate the
 * reduced auxiliary problem (exactly affine here: c(mu)), then F_mu, its
 * inverse and det at every ECM point (Sec. 3.4); cache F_mu^-1 and
 * w_q |det F_mu|.  Sets r = 0 and the virgin history (F^pl = I, xi = 0,
 * Appendix A).
 *   mu_dev    : f64 [batch][n_mu] device; read only.
 *   state_dev : rom_state_bytes(h, batch) bytes of device memory.
 * Synchronises `stream`.  Returns ROM_EINVAL_MU if any point has
 * det F_mu <= 0 at an ECM point; such points get status ROM_ST_BADMU from
 * rom_step and are never solved.  The other points are initialised normally.
 */
int rom_state_init(rom_handle h, int32_t batch, const double* mu_dev, void* state_dev, hipStream_t stream);

/*
 * rom_step -- Algorithm 1 online, step 2: Newton on the reduced coordinates
 * (eq. red_newton) with the hyper-reduced force and stiffness
 * (eqs. forcevector_ecm, stiffnessmatrix_ecm), from the committed state to
 * the macroscopic deformation gradient Fbar (absolute, not an increment),
 * then steps 3-5: effective stress and stiffness (eqs. eff_stress_1,
 * tangent_problem_red, eff_stiffness_1) at the returned state, stored in the
 * state.
 *   Fbar_dev   : f64 [batch][4] device, in-plane Fbar (Fbar_33 = 1).
 *   opts       : host pointer; NULL means rom_default_opts.
 *   status_dev : i32 [batch] device out, ROM_ST_*.
 *   iters_dev  : i32 [batch] device out, Newton evaluations made.
 *   resnorm_dev: f64 [batch] device out, ||f||_2 at the returned state.
 * The trial r and history are always written; they replace the committed
 * ones only where opts->commit is set and the point converged, so a failed
 * point can be retried with a smaller load step (Appendix A).
 */
int rom_step(rom_handle h, int32_t batch, const double* Fbar_dev, void* state_dev,
             const rom_opts* opts, int32_t* status_dev, int32_t* iters_dev,
             double* resnorm_dev, hipStream_t stream);

/*
 * rom_homogenized_stress_tangent -- effective stress Pbar (eq. eff_stress_1)
 * and stiffness Abar (eqs. eff_stiffness_1, eff_stress_f11) of the last
 * rom_step on this state; Abar uses K* = K at the returned state
 * (Sec. 3.3).  Normalised by the cell area.
 *   Pbar_dev : f64 [batch][4] device out.
 *   Abar_dev : f64 [batch][16] device out, row (ij) column (kl).
 */
int rom_homogenized_stress_tangent(rom_handle h, int32_t batch, const void* state_dev,
                                   double* Pbar_dev, double* Abar_dev, hipStream_t stream);

/*
 * rom_commit_trial -- commit the trial state left by the last rom_step on
 * this state, a step made with opts.commit = 0 to Fbar_dev: where status_dev
 * reports convergence (ROM_ST_CONVERGED or ROM_ST_FALLBACK) the trial r, the
 * trial history and Fbar become the committed ones, the internal variables
 * of the last converged load step from which the next one starts
 * (Appendix A).  The state is then the one a step with opts.commit = 1 to the
 * same Fbar from the same committed state leaves (the same Newton map from
 * the same start).  The two-scale loop (Sec. 4.2) commits the RVE solves of
 * its converged macro iteration this way instead of solving them again.
 * Other points keep their committed state.  Asynchronous on `stream`.
 *   Fbar_dev   : f64 [batch][4] device, the load of that step.
 *   status_dev : i32 [batch] device, the statuses that step returned.
 * The trial step must have been made without load-step cutting (cutting
 * commits its converged sub-steps in place, so it runs with commit only).
 */
int rom_commit_trial(rom_handle h, int32_t batch, const double* Fbar_dev, void* state_dev,
                     const int32_t* status_dev, hipStream_t stream);

/*
 * rom_step_noalloc -- for callers that cannot allocate device memory or
 * create runtime objects during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  The same solve as
 * rom_step with opts->mode = ROM_MODE_FUSED on a persistent grid
 * (opts->grid_per_cu workgroups per compute unit, 0 meaning 2), same
 * arguments and the same results bit for bit; the work list and queue
 * counters of the persistent grid live in a static device array of the
 * library (ROM_NOALLOC_MAX_BATCH + 64 int32, 128.25 KiB per device, held
 * until the process ends) instead of the state, and no timing marks are
 * recorded.  The call allocates nothing and creates no event.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other threads, other handles) race and must be
 * serialised by the caller.  The counters are cleared by a kernel at the
 * start of each call, so the array's previous contents do not matter.
 * Errors: as rom_step; ROM_ESCRATCH when batch > ROM_NOALLOC_MAX_BATCH;
 * ROM_EUNSUPPORTED for another mode; ROM_EHIP when the array's device
 * address was not found at rom_load.
 */
#define ROM_NOALLOC_MAX_BATCH 32768
int rom_step_noalloc(rom_handle h, int32_t batch, const double* Fbar_dev, void* state_dev,
                     const rom_opts* opts, int32_t* status_dev, int32_t* iters_dev,
                     double* resnorm_dev, hipStream_t stream);

/*
 * rom_shape_sensitivity -- sensitivities of the effective stress to the shape
 * parameters, dPbar/dmu (eq. eff_sensitivities_full with the ECM rule), at
 * the returned state of the last rom_step on this state, with the committed
 * history held fixed: call it after a step made with opts.commit = 0 (a
 * trial solve; the committed history is then the one the step started from),
 * with the same Fbar.  The fluctuation's share follows from the reduced
 * equilibrium, dr/dmu = -K*^-1 df/dmu, using the K*^-1 C the step kept (the
 * consistent tangent is symmetric).  Asynchronous on `stream`.
 *   Fbar_dev  : f64 [batch][4] device, the load of that step.
 *   dPdmu_dev : f64 [batch][4][n_mu] device out, component (iJ) of Pbar by
 *               shape parameter (in the order of rom_state_init's mu); NaN for
 *               points whose mu was rejected.
 * Returns ROM_EUNSUPPORTED when n * n_mu > 1024.
 */
int rom_shape_sensitivity(rom_handle h, int32_t batch, const double* Fbar_dev, const void* state_dev,
                          double* dPdmu_dev, hipStream_t stream);

/*
 * Learned warm start.  A fully connected network (n_in -> 3 hidden layers of
 * `width` SiLU units -> n_out) predicts the Newton increment of the reduced
 * coordinates of a load step, dr = r_converged - r_committed, from per-point
 * features (rom_features).  Weights are kept as an FP32 master copy with BF16
 * copies for the BF16 forward; training runs the library's own forward,
 * backward (FP32) and Adam kernels.  With opts.warm_start = ROM_WARM_MLP,
 * rom_step starts Newton from r_committed + dr and falls back to the plain
 * guess when ||f|| has not dropped tenfold after two Newton updates
 * (status ROM_ST_FALLBACK when it then converges).  Newton judges the guess:
 * a point is converged only at ||f||_2 <= tol, so where a step is solved
 * over the same (sub-)steps as from the plain guess (equal
 * ROM_FIELD_SUBSTEPS records) the two results differ only within the
 * tolerance.  With load-step cutting a better guess can let a full step
 * converge that the plain guess would cut into sub-steps (or the reverse);
 * the point then integrates its plastic flow over other increments, a
 * different loading path of its own history.
 *
 * Parameter layout (FP32, host): W1 [n_in][width], b1 [width], W2 [width][width],
 * b2, W3 [width][width], b3, W4 [width][n_out], b4 [n_out].
 * Precision arguments: ROM_DT_F32 or ROM_DT_BF16 (forward); backward is FP32.
 */
int rom_mlp_create(int32_t n_in, int32_t width, int32_t n_out, int32_t max_batch, int device, rom_mlp_handle* out);
int rom_mlp_free(rom_mlp_handle m);
int rom_mlp_param_count(rom_mlp_handle m, int64_t* count);
int rom_mlp_set_params(rom_mlp_handle m, const float* host_params, int64_t count);
int rom_mlp_get_params(rom_mlp_handle m, float* host_params, int64_t count);
/* affine scaling of features and targets: x_hat = (x - x_mean) / x_std, y = y_mean + y_std * y_hat (host arrays) */
int rom_mlp_set_scaling(rom_mlp_handle m, const float* x_mean, const float* x_std, const float* y_mean,
                        const float* y_std);
/* raw features X [batch][n_in] (device) -> raw predictions Y [batch][n_out] (device) */
int rom_mlp_forward(rom_mlp_handle m, int32_t batch, const float* X_dev, float* Y_dev, int32_t precision,
                    hipStream_t stream);
/* loss = mean over the batch of sum (y_hat - (Y - y_mean) / y_std)^2, and its parameter gradient
   (same layout as the parameters) into grads_dev (device, may be NULL) */
int rom_mlp_gradients(rom_mlp_handle m, int32_t batch, const float* X_dev, const float* Y_dev, int32_t precision,
                      float* grads_dev, float* loss_dev, hipStream_t stream);
/* gradients as above, then one Adam update (beta1 0.9, beta2 0.999, eps 1e-8, step counter kept inside) */
int rom_mlp_train_step(rom_mlp_handle m, int32_t batch, const float* X_dev, const float* Y_dev, float lr,
                       int32_t precision, float* loss_dev, hipStream_t stream);
/* rom_mlp_infer: the network's inference on raw features (the same call as rom_mlp_forward) */
int rom_mlp_infer(rom_mlp_handle m, int32_t batch, const float* X_dev, float* Y_dev, int32_t precision,
                  hipStream_t stream);
/* One epoch of minibatch Adam over N samples X [N][n_in], Y [N][n_out] (device): minibatch j takes the
   rows order[j * batch .. (j + 1) * batch - 1] (device i32 [N], a permutation chosen by the caller),
   floor(N / batch) updates at learning rate lr; loss_sum_dev (device f32) receives the sum of the
   minibatch losses.  batch <= max_batch. */
int rom_mlp_train_epoch(rom_mlp_handle m, int32_t N, const float* X_dev, const float* Y_dev, const int32_t* order_dev,
                        int32_t batch, float lr, int32_t precision, float* loss_sum_dev, hipStream_t stream);
/* Scaling from N >= 2 samples (device): the column means and standard deviations (N - 1 in the
   denominator, 1 for a column whose deviation is below 1e-12) of X and Y become x_mean, x_std,
   y_mean, y_std.  FP64 accumulation, enqueued on `stream`. */
int rom_mlp_fit_scaling(rom_mlp_handle m, int32_t N, const float* X_dev, const float* Y_dev, hipStream_t stream);
/* Network artifact (host memory): "PODECMN1", u32 version 1, n_in, width, n_out, u32 0, then f32
   x_mean, x_std, y_mean, y_std and the parameters in the layout above.  rom_mlp_save writes it when
   blob is non-NULL and capacity suffices (*bytes: its size; synchronises the device); rom_mlp_load
   creates a network from it (errors as rom_load: ROM_EFORMAT for a bad magic, size, non-finite value
   or a deviation <= 0, ROM_EVERSION). */
int rom_mlp_save(rom_mlp_handle m, void* blob, size_t capacity, size_t* bytes);
int rom_mlp_load(const void* blob, size_t bytes, int32_t max_batch, int device, rom_mlp_handle* out);

/*
 * rom_features -- per-point inputs of the warm-start network for the step
 * to Fbar_dev: mu (n_mu), Fbar - Fbar_committed (4), r_committed (n), and eight
 * statistics of the committed plastic state weighted by w_q |det F_mu|
 * (mean, max and standard deviation of xi, the yielded fraction, the mean of
 * F^pl - I).  X_dev: f32 [batch][n_mu + 4 + n + 8] device out.
 */
int rom_features(rom_handle h, int32_t batch, const double* Fbar_dev, const void* state_dev, float* X_dev,
                 hipStream_t stream);

/*
 * rom_warm_samples -- training samples of the warm-start network from the
 * load step just solved on this state: for every point whose status_dev
 * entry is ROM_ST_CONVERGED, in point order, its features X_feat_dev
 * [batch][n_in] (rom_features before the step) and its increment
 * dr = r_committed - r_before_dev (r_before_dev: f64 [batch][n], the
 * committed r before the step) in FP32, written at rows *count_dev,
 * *count_dev + 1, ... of X_out_dev [.][n_in] and Y_out_dev [.][n]; *count_dev
 * (device i32) is advanced.  The caller sizes the outputs for every sample
 * it collects.  Asynchronous on `stream`.
 */
int rom_warm_samples(rom_handle h, int32_t batch, const void* state_dev, const float* X_feat_dev,
                     const double* r_before_dev, const int32_t* status_dev, float* X_out_dev, float* Y_out_dev,
                     int32_t* count_dev, hipStream_t stream);

/*
 * Uneven batches: every point p follows its own path of nsteps[p] load steps
 * (paths_dev: f64 [batch][max_steps][4]).  rom_path_gather sets, for the
 * points with step[p] < nsteps[p], Fbar[p] = paths[p][step[p]] and
 * active[p] = 1 (else active[p] = 0, Fbar[p] unchanged); rom_path_advance
 * increments step[p] where active[p].  With rom_step(opts.active = active),
 * a whole load step of the batch is device-driven and can be captured once
 * in a HIP graph and replayed (no allocation, memset or synchronisation).
 */
int rom_path_gather(int32_t batch, const double* paths_dev, int32_t max_steps, const int32_t* nsteps_dev,
                    const int32_t* step_dev, double* Fbar_dev, int32_t* active_dev, hipStream_t stream);
int rom_path_advance(int32_t batch, const int32_t* active_dev, int32_t* step_dev, hipStream_t stream);

/*
 * Measurement support.  While enabled, rom_step records a HIP event pair on
 * the caller's stream around every launch of its dominant kernel (the
 * reduced-tangent contraction of eq. stiffnessmatrix_ecm in the staged form;
 * the whole Newton kernel in the fused form).  rom_timing_read waits for the
 * recorded events and returns the summed kernel time and the number of
 * launches since the last enable; it is meant for benchmarks, not hot loops.
 */
int rom_timing_enable(rom_handle h, int enable);
int rom_timing_read(rom_handle h, double* total_ms, int64_t* launches);

/*
 * Two-scale (FE^2) macro side (Sec. 4.2: a block of eight-node quadrilateral
 * elements with four Gauss points each, fixed where the caller says,
 * loaded on its top edge by the downward traction
 * T(x) = Tbar (1 - (2 x / W - 1)^2) as a dead load).  Its quadrature points
 * p = 4 e + g (g: Gauss points (-,-), (+,-), (+,+), (-,+) of the parent
 * square) are the batch of rom_step: Fbar from the macro displacements,
 * then Pbar and Abar of the RVE back into the macro Newton step.  Total
 * Lagrangian, plane strain; dofs 2 n + i.
 *
 * rom_fe2_create copies the mesh (host arrays): X [nodes][2]; conn
 * [elements][8], corners counterclockwise from the parent corner (-1, -1),
 * then the midsides of the bottom, right, top and left edges; the fixed
 * dofs; top [ntop][3] the nodes of each loaded edge (ends and middle, in
 * order along the edge); width W of the traction profile.  It computes the
 * point geometry on the device and sizes the banded solve from the
 * numbering (half-bandwidth kl of the free dofs at most 255: number the
 * nodes across the short side).  Returns ROM_EINVAL for out-of-range
 * indices, repeated fixed dofs or no free dof, ROM_EUNSUPPORTED for a wider
 * band.  The handle owns the band workspace: calls that overlap on one
 * handle race.  All other buffers are caller-owned device memory; the calls
 * enqueue on the stream and do not synchronise.
 *
 * rom_fe2_gradient:   Fbar[p][4] = I + sum_a u_a (x) dN_a/dX.
 * rom_fe2_traction:   fext[dofs], the consistent nodal forces of T(x).
 * rom_fe2_residual:   res[dofs] = fext - sum_p B_p^T Pbar_p w|J|; if norms is
 *                     given, norms[0..1] = ||res||_2, ||fext||_2 over the
 *                     free dofs.
 * rom_fe2_solve:      assembles K_ff = sum_p B^T Abar_p B w|J| (free rows and
 *                     columns) and solves K_ff du_f = res_f - K_fd du_d by
 *                     banded LU with partial pivoting; u_f += du_f and
 *                     u_d += du_d (du_d [nfixed] in the order of the fixed
 *                     list, or NULL for zero).  info = 0, or k + 1 when
 *                     column k has no nonzero pivot (u unchanged).
 * rom_fe2_compliance: C = int_top T(x) (-u_y) dx, the work of the load.
 */
typedef struct rom_fe2* rom_fe2_handle;
int rom_fe2_create(int32_t nodes, int32_t elements, const double* X_host, const int32_t* conn_host, int32_t nfixed,
                   const int32_t* fixed_dofs_host, int32_t ntop, const int32_t* top_host, double width, int device,
                   rom_fe2_handle* out);
int rom_fe2_free(rom_fe2_handle h);
int rom_fe2_info(rom_fe2_handle h, int32_t* dofs, int32_t* free_dofs, int32_t* points, int32_t* kl);
int rom_fe2_points(rom_fe2_handle h, double* Xg_dev, hipStream_t stream);
int rom_fe2_gradient(rom_fe2_handle h, const double* u_dev, double* Fbar_dev, hipStream_t stream);
int rom_fe2_traction(rom_fe2_handle h, double Tbar, double* fext_dev, hipStream_t stream);
int rom_fe2_residual(rom_fe2_handle h, const double* Pbar_dev, const double* fext_dev, double* res_dev,
                     double* norms_dev, hipStream_t stream);
int rom_fe2_solve(rom_fe2_handle h, const double* Abar_dev, const double* res_dev, const double* dud_dev,
                  double* u_dev, int32_t* info_dev, hipStream_t stream);
int rom_fe2_compliance(rom_fe2_handle h, double Tbar, const double* u_dev, double* C_dev, hipStream_t stream);

/*
 * Offline stage: POD by the method of snapshots (Sec. 3.1, the fluctuation
 * modes of eq. pod_disp in the V^p inner product; Sec. 3.2, the weighted-
 * stress modes in L^2 of the parent domain).  Snapshots S_dev [ns][nrow]
 * (snapshot j contiguous); the weight M, symmetric positive definite, given
 * either as a diagonal mdiag_dev [nrow] or as a CSR matrix (csr_ptr [nrow +
 * 1], csr_col, csr_val), exactly one of the two.  Computes C = S^T M S, its
 * eigenvalues lambda_dev [ns] (descending) and the n leading modes
 * phi_k = S v_k / sqrt(lambda_k), re-orthonormalised once in the M product
 * (phi <- phi L^-T, L L^T = phi^T M phi), into modes_dev [n][nrow] (mode k
 * contiguous; the sign of each mode is that of the eigensolver's vector).
 * work_dev: rom_pod_workspace(nrow, ns, n) bytes of device memory.  The
 * call synchronises the stream (the rank test reads the eigenvalues) and
 * the eigensolver and Cholesky steps may allocate their own scratch.
 * Returns ROM_EINVAL when n exceeds the numerical rank (eigenvalues above
 * 1e-13 of the largest) or the arguments are inconsistent, ROM_EHIP when
 * a device step fails.
 */
int rom_pod_workspace(int32_t nrow, int32_t ns, int32_t n, size_t* bytes);
int rom_pod(int32_t nrow, int32_t ns, const double* S_dev, const double* mdiag_dev, const int32_t* csr_ptr_dev,
            const int32_t* csr_col_dev, const double* csr_val_dev, int32_t n, double* modes_dev, double* lambda_dev,
            void* work_dev, size_t work_bytes, hipStream_t stream);

/*
 * Offline stage: empirical cubature (Sec. 3.2, eqs. integralsbasis and
 * integral_ecm) by the greedy of the published method the paper defers to.
 * Integrands J_dev [R][nq] (integrand i at quadrature point q) with full
 * rule weights w_dev [nq] (positive).  J diag(sqrt(w)) = U Sigma V^T, rank r
 * (singular values above 1e-12 of the largest), Z = V_r^T diag(1/sqrt(w)),
 * b = Z w; from an empty set and res = b, repeatedly: the point of largest
 * positive Z_q . res / |Z_q| (lowest index on ties) joins, least squares on
 * the selected set (non-negative least squares when a weight is not
 * positive), points of zero weight leave, res = b - Z_S w_S; until
 * |res| <= eps |b|, m_max points or 10 m_max iterations, or no positive
 * correlation is left.  Outputs: the selected points in selection order
 * idx_dev [m_max] and their weights weights_dev [m_max], their count *m_out;
 * optionally |res| / |b| after each iteration (hist_host, host memory,
 * starting with 1, at most hist_cap entries, count *hist_len) and the rank r.
 * m_max <= 1024.  work_dev: rom_ecm_workspace(R, nq, m_max) bytes.  The call
 * synchronises the stream once per iteration (the stop test) and the SVD
 * step may allocate its own scratch.  Returns ROM_EUNSUPPORTED (results so
 * far written) if a chosen column is linearly dependent on the selected ones.
 */
int rom_ecm_workspace(int32_t R, int32_t nq, int32_t m_max, size_t* bytes);
int rom_ecm(int32_t R, int32_t nq, const double* J_dev, const double* w_dev, double eps, int32_t m_max,
            int32_t* idx_dev, double* weights_dev, int32_t* m_out, double* hist_host, int32_t hist_cap,
            int32_t* hist_len, int32_t* rank_out, void* work_dev, size_t work_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
