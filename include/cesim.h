/*
 * cesim.h -- C ABI of the MI355X (gfx950) library for conditional simulation
 * of a stationary Gaussian field by circulant embedding, extended to
 * irregularly spaced observations by local Kriging.
 *
 * Method: Bailey, Bandyopadhyay and Nychka, "Adapting conditional simulation
 * using circulant embedding for irregularly spaced spatial data"
 * (arXiv 2109.11044).  Section numbers below refer to that paper.
 *
 * Call sequence for one event (one covariance model, grid and data set):
 *
 *   ce_setup        -- circulant-embedding eigenvalues of the torus
 *                      covariance (Section 1; Section 2.1 item (a)).
 *   offgrid_nnkrige -- local-Kriging weights and conditional variances of
 *                      the off-grid observations from their (2 n_p)^2
 *                      nearest grid nodes (Section 2.1 items (b)-(c);
 *                      Section 3.1; Section 3.6).
 *   ce_simulate     -- unconditional grid realizations y_r by the CE draw
 *                      (step 2 of the algorithm in Section 2).
 *   condition       -- synthetic observations z*_r (step 3 under local
 *                      Kriging), Kriging of z - z*_r onto the grid with the
 *                      plain nugget (steps 1, 4, 5 and item (d); eq. (4) of
 *                      Section 3), in place:
 *                          v_r = y_r + K12 (K22 + tau^2 I)^{-1} (z - z*_r).
 *   ce_destroy
 *
 * ce_simulate and condition may be repeated for further batches of
 * realizations; condition always applies to the batch the last ce_simulate
 * produced.
 *
 * Conventions
 *   - Every entry point returns a cesim_status; nothing throws or aborts
 *     across the ABI.  cesim_status_string() names a status.
 *   - The context owns every internal device buffer.  The caller owns the
 *     host input arrays (copied before the call returns) and the device
 *     field buffers it passes in.
 *   - Work is enqueued on the HIP stream given to ce_setup (NULL = the
 *     default stream).  ce_simulate, and condition() when the factor of
 *     the observation covariance is current, return once their work is
 *     queued; a condition() call that (re)factorises waits for the
 *     factorisation (not for the grid product) to return its status.  The
 *     calls documented below as synchronising (ce_setup, offgrid_nnkrige,
 *     ce_get_info, ce_grad_linear, ce_grad_vjp, ce_prediction_se, nn_surrogate, the
 *     batch and tuning calls, the stage times) wait for their work.  A
 *     context also owns two internal streams (default priority), ordered
 *     with the given stream by events; ce_destroy drains them.
 *   - Use a context from one host thread at a time.
 *   - Fields are stored [r][j][i]: realization, grid row (y), grid column
 *     (x, fastest).  Grid node (i, j) sits at (x0 + i dx, y0 + j dy).
 *   - Random numbers: Philox4x32-10 keyed by the 64-bit seed; realization r
 *     depends only on (seed, r), never on how realizations were batched.
 *
 * Precision (cesim_precision)
 *   CESIM_PREC_FP64  : every step in FP64; fields are double.
 *   CESIM_PREC_MIXED : eigenvalue setup, local-Kriging solves, the
 *                      observation Cholesky and its solves in FP64; the CE
 *                      FFT passes in FP32; the cross-covariance product
 *                      K12 B on matrix cores in half precision (FP16 by
 *                      default, BF16 selectable) with FP32 accumulation and
 *                      a three-product split-precision correction; fields
 *                      are float.
 */
#ifndef CESIM_H
#define CESIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cesim_ctx_s* cesim_ctx;

typedef enum {
  CESIM_OK = 0,
  CESIM_ERR_INVALID_ARG = 1,        /* argument out of range or NULL        */
  CESIM_ERR_NEGATIVE_EIGENVALUE = 2,/* no admissible torus on the ladder    */
  CESIM_ERR_NOT_POSITIVE_DEFINITE = 3, /* a Cholesky factorisation failed   */
  CESIM_ERR_OBS_OUTSIDE_GRID = 4,   /* an observation lies outside the grid */
  CESIM_ERR_OUT_OF_MEMORY = 5,      /* device allocation failed             */
  CESIM_ERR_HIP = 6,                /* a HIP runtime call failed            */
  CESIM_ERR_BAD_STATE = 7           /* call out of order                    */
} cesim_status;

typedef enum { CESIM_PREC_FP64 = 0, CESIM_PREC_MIXED = 1 } cesim_precision;

/* Matern covariance (Section 3.3):
 *   C(h) = sigma2 * 2^(1-nu)/Gamma(nu) * (sqrt(2 nu) d/range)^nu
 *                 * K_nu(sqrt(2 nu) d/range),
 * with d the anisotropic lag length sqrt(u^2 + aniso_ratio^2 w^2), where
 * (u, w) is the lag rotated by -aniso_angle (range along aniso_angle,
 * range/aniso_ratio across it).  nu must be 0.5, 1.0 or 1.5;
 * sigma2 > 0; range > 0; aniso_ratio >= 1. */
typedef struct {
  double nu;
  double sigma2;
  double range;
  double aniso_ratio;
  double aniso_angle;
} cesim_cov;

/* Regular m1 x m2 grid with spacing (dx, dy) > 0 and origin (x0, y0).
 * t1, t2: torus size; 0 chooses it by the ladder S(f m) for
 * f = 2, 3, 4, 6, 8 (S(n): smallest 2^a 3^b 5^c >= n), the first with
 * min eigenvalue >= -1e-12 max eigenvalue.  A forced size must be
 * >= 2 m - 1 on each axis, a product of 2, 3 and 5, and at most 8192. */
typedef struct {
  int m1, m2;
  double x0, y0, dx, dy;
  int t1, t2;
} cesim_grid;

typedef struct {
  int t1, t2;                 /* torus actually used                      */
  double lam_min, lam_max;    /* eigenvalue extremes of the accepted torus*/
  double lam_sum;             /* sum of eigenvalues = t1 t2 C(0)          */
  double max_imag;            /* largest |Im| of the spectrum             */
  int nobs, k;                /* observations and window size             */
  double gamma_min, gamma_max;/* local-Kriging conditional variances      */
  double ms_setup;            /* last ce_setup wall time (ms)             */
  double ms_offgrid;          /* last offgrid_nnkrige (ms, enqueue only)  */
  int precision;              /* cesim_precision                          */
  int torus_tries;            /* ladder entries evaluated                 */
} cesim_info;

/* Circulant-embedding setup (Section 1; Section 2.1 item (a)).
 * Builds the torus base c[q2][q1] = C(w(q1) dx, w(q2) dy) in FP64
 * (w(q) = q for q <= T/2, else q - T; on Nyquist lines the two signs of
 * that lag component are averaged), its 2D FFT in FP64 on the GPU, and
 * checks min(lambda) >= -1e-12 max(lambda) in FP64; tiny negatives are
 * clamped to 0 and sqrt(lambda) is kept in FP64 (and FP32 for
 * CESIM_PREC_MIXED).  hip_stream: a hipStream_t or NULL.  On success *out
 * owns a new context.  Errors: INVALID_ARG, NEGATIVE_EIGENVALUE (ladder
 * exhausted or forced torus rejected; no context is created),
 * OUT_OF_MEMORY, HIP.  Synchronises the stream. */
cesim_status ce_setup(const cesim_cov* cov, const cesim_grid* grid,
                      cesim_precision prec, void* hip_stream,
                      cesim_ctx* out);

/* Unconditional draw of nreal realizations, absolute indices first_real ..
 * first_real + nreal - 1 (step 2 of Section 2; Section 2.1 item (a)), two
 * per transform: realizations 2P and 2P + 1 form pair P and
 *   W_P = FFT2(sqrt(lambda / N) (eps_{2P} + i eps_{2P+1})),  N = t1 t2,
 *   y_{2P} = Re W_P[0:m2, 0:m1],  y_{2P+1} = Im W_P[0:m2, 0:m1],
 * eps_r the t2 x t1 torus noise of Philox stream 0 (element q = j t1 + i:
 * block q/4, word q%4, counter (block, r, event id, 0), Box-Muller).  The
 * real and imaginary parts are independent fields of covariance C
 * (lambda is real and even).  Pairs are absolute, so y_r depends only on
 * (seed, r); a call that starts or ends inside a pair transforms the whole
 * pair and writes its own member.  fields_dev: caller-owned
 * device buffer of nreal*m2*m1 doubles (FP64) or floats (MIXED), written
 * asynchronously.  Records (seed, first_real, nreal) for condition().
 * Errors: INVALID_ARG (nreal < 1, first_real < 0, NULL), OUT_OF_MEMORY,
 * HIP. */
cesim_status ce_simulate(cesim_ctx ctx, int nreal, uint64_t seed,
                         int first_real, void* fields_dev);

/* ce_simulate for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same draw, bit for bit, with its pair buffers in a static device array of
 * 64 MiB instead of memory the context allocates.  The library holds one
 * such array on every device it runs on, until the process ends; its
 * address is looked up once per device by ce_setup.  Pairs are processed in
 * chunks that fit it (the buffer of one pair is 8 t1 m2 bytes on MIXED,
 * 16 t1 m2 on FP64).  Every call on a device shares that device's array:
 * calls that overlap on one device (on different streams or contexts) race
 * and must be ordered by the caller.  The call allocates nothing and calls
 * no allocating routine; stage timing is off for it.  Arguments, fields_dev
 * ownership and the record kept for condition() as for ce_simulate.
 * Errors: INVALID_ARG (as ce_simulate, or one pair's buffer larger than
 * 64 MiB), BAD_STATE (no array address), HIP. */
cesim_status ce_simulate_noalloc(cesim_ctx ctx, int nreal, uint64_t seed,
                                 int first_real, void* fields_dev);

/* Local-Kriging setup (Section 2.1; Section 3.1; Section 3.6).
 * obs_xy_host: nobs (x, y) pairs, host memory, copied.  k = (2 n_p)^2 in
 * {4, 16, 36, 64} and 2 n_p <= min(m1, m2).  Window of s: lower-left node
 * a = clamp(floor((sx - x0)/dx) - n_p + 1, 0, m1 - 2 n_p), likewise b;
 * nodes (a+p, b+q), index q*2n_p + p.  Computes in FP64 the Cholesky factor
 * of the window covariance K11 (identical for every window) and per
 * observation w_i = K11^{-1} k_i and gamma_i = C(0) - k_i . w_i (>= 0).
 * Errors: INVALID_ARG, OBS_OUTSIDE_GRID (any point outside
 * [x0, x0 + (m1-1) dx] x [y0, y0 + (m2-1) dy], widened by 1e-12 of the
 * extent for rounding, or not finite),
 * NOT_POSITIVE_DEFINITE (K11), OUT_OF_MEMORY, HIP.  Invalidates the
 * factorisation held for condition() and ends the nearest-neighbour mode
 * of nn_surrogate.  Synchronises. */
cesim_status offgrid_nnkrige(cesim_ctx ctx, int nobs, const double* obs_xy_host,
                             int k);

/* Conditioning (steps 1, 3, 4, 5 of Section 2 with items (c), (d) of
 * Section 2.1; eq. (4) of Section 3), in place on the batch last produced
 * by ce_simulate into fields_dev (the same buffer and type):
 *   z*_{r,i} = w_i . y_r[window_i] + sqrt(nugget + gamma_i) xi_{r,i}
 *       (xi from Philox stream 1: block i/4, word i%4, counter
 *        (block, r, event id, 1)),
 *   B_r     = (K22 + nugget I)^{-1} (z - z*_r)        (FP64 Cholesky),
 *   v_r     = y_r + K12 B_r,  K12[g, i] = C(g - s_i).
 * MIXED evaluates v_r as y_r + yhat - K12 (K22 + nugget I)^{-1} z*_r with
 * the prediction yhat = K12 (K22 + nugget I)^{-1} z computed once in FP64
 * (kept while the factor and z are unchanged) and the per-realization
 * product in the half-precision split GEMM.
 * z_host: nobs observed values, host memory, copied.  nugget >= 0.  The
 * Cholesky factor of K22 + nugget I is kept and reused while the nugget and
 * the observation set are unchanged.  MIXED, on a reused factor of at most
 * 8192 stations, with at most 128 realizations: B_r comes from one FP64
 * GEMM with (K22 + nugget I)^{-1}, formed on the first such call and kept
 * with the factor (n^2 doubles), instead of the blocked substitutions (the
 * same coefficients up to FP64 rounding).  A batch is conditioned once: after a
 * successful call the next condition() needs a new ce_simulate (the fields
 * are conditional now).  After NOT_POSITIVE_DEFINITE the fields are
 * unchanged and the batch may be conditioned again (e.g. with another
 * nugget).  Errors: BAD_STATE (no offgrid_nnkrige, or no ce_simulate since
 * the last successful condition), INVALID_ARG, NOT_POSITIVE_DEFINITE,
 * OUT_OF_MEMORY, HIP. */
cesim_status condition(cesim_ctx ctx, const double* z_host, double nugget,
                       void* fields_dev);

/* Statistics of the context; synchronises the stream. */
cesim_status ce_get_info(cesim_ctx ctx, cesim_info* info);

/* Copies sqrt(lambda / (t1 t2)) (FP64, t2 x t1, row-major) -- the spectral
 * multiplier the draw applies -- into a caller-owned device buffer. */
cesim_status ce_copy_spectrum(cesim_ctx ctx, double* dev_out);

/* Copies the local-Kriging results of the last offgrid_nnkrige into
 * caller-owned device buffers (any may be NULL): window corners as int32
 * pairs (a, b) [nobs][2], weights [nobs][k] FP64, gamma [nobs] FP64. */
cesim_status offgrid_copy_weights(cesim_ctx ctx, int* corners_dev,
                                  double* weights_dev, double* gamma_dev);

/* Copies the Kriging coefficients B_r = (K22 + nugget I)^{-1} (z - z*_r) of
 * the last condition() call ([nreal][nobs] FP64) into a caller-owned device
 * buffer. */
cesim_status condition_copy_coefficients(cesim_ctx ctx, double* dev_out);

/* Host evaluation of the library's covariance code (the same source the
 * kernels run) at n lags (hx[i], hy[i]) into out[i], FP64.  For tests. */
cesim_status cesim_covariance_host(const cesim_cov* cov, int n,
                                   const double* hx, const double* hy,
                                   double* out);

/* Host evaluation of the library's Philox4x32-10 (same source as the
 * kernels): out[4*i .. 4*i+3] = words of counter (ctr0[i], c1, c2, c3). */
cesim_status cesim_philox_host(uint64_t seed, int n, const uint32_t* ctr0,
                               uint32_t c1, uint32_t c2, uint32_t c3,
                               uint32_t* out);

const char* cesim_status_string(cesim_status s);

/* ---- instrumentation and memory (not part of the method) ----
 * Stage timing: when enabled, the library records a pair of HIP events on
 * the context's stream around each stage it launches (per launch or per
 * chunk of launches); times accumulate until read with reset != 0.
 * Stages, in order (CESIM_NUM_STAGES of them): torus base, setup FFT,
 * eigenvalue check, draw pass A (pair noise, scaling, column FFT), draw
 * pass B (row FFT + crop),
 * local-Kriging setup, observation Cholesky, synthetic observations and
 * right-hand sides, observation solves, half-precision split of the
 * coefficients, cross-covariance GEMM onto the grid, FP64 prediction from the
 * observed values (MIXED only; with its one-vector solve A^{-1} z); for
 * ce_prediction_se: W1 K11 W1^T, the
 * covariance rows of a chunk of grid nodes (K12 and (W1 K11)^T), the GEMM of
 * the solved rows with W1 K11 W1^T, and the per-node reduction. */
#define CESIM_NUM_STAGES 16

/* Launch-shape parameters (performance only; results do not change):
 *   CESIM_PARAM_GEMM_TILE: workgroup tile of the mixed cross-covariance GEMM,
 *     1 = 128 grid nodes x 256 realizations (4 waves), 2 = 256 x 256 (4 waves
 *     of two 32-node fragments), 3 = 128 x 512 (8 waves; the correlations of
 *     each observation chunk are computed once for all 512 realizations),
 *     4 = 128 x 64 and 5 = 128 x 128 (calls of few realizations: no matrix
 *     work on padding); 0 (default) takes the tuning table's choice for the
 *     problem's shape, else 1.  Tiles 1, 2, 4 and 5 skip the observation
 *     chunks whose correlations with their nodes all round to zero in the
 *     FP16 split (products that are exact zeros), so the fields do not
 *     depend on the tile.
 *   CESIM_PARAM_DRAW_COLS, CESIM_PARAM_DRAW_ROWS: torus columns per
 *     workgroup of draw pass A and grid rows per workgroup of pass B on the
 *     register-FFT path (square tori of 2^a from 128 to 8192 and of 3 * 2^a
 *     from 384 to 6144); powers of two, clamped to each kernel's largest
 *     shape; 0 (default) takes the tuning table's choice, else the largest.
 *   CESIM_PARAM_DRAW_CHUNK_PAIRS: realization pairs per launch of the draw
 *     passes (bounds the pair buffer); 0 (default) chooses up to 2 GiB.
 *   CESIM_PARAM_GEMM_SPLIT (changes rounding, not the method): arithmetic
 *     of the mixed path's cross-covariance product, 0 = FP16 three-product
 *     split (default, about 22 significant bits per operand), 1 = BF16
 *     three-product split (about 16 bits), 2 = plain FP32 on matrix cores
 *     (24 bits, no split; the comparison variant, 3x the issued time of the
 *     split at the FP32 matrix rate). */
#define CESIM_PARAM_GEMM_TILE 1
#define CESIM_PARAM_DRAW_CHUNK_PAIRS 2
#define CESIM_PARAM_GEMM_SPLIT 3
/*   CESIM_PARAM_EVENT_ID (changes the realizations): word 2 of the Philox
 *     counter of the torus noise and of xi, >= 0 (default 0); a context with
 *     event id e draws exactly what event e of a batch draws. */
#define CESIM_PARAM_EVENT_ID 4
#define CESIM_PARAM_DRAW_COLS 6
#define CESIM_PARAM_DRAW_ROWS 7
/*   CESIM_PARAM_JOINT_BOXES (changes the method, Section 2.1 last paragraph
 *     and Section 3.6): 1 draws the synthetic values of observations that
 *     share a grid box (the cell floor((x - x0)/dx), floor((y - y0)/dy))
 *     jointly from their conditional law given the box's window,
 *     z*_G = W1_G y + L_G xi_G with L_G L_G^T = tau^2 I + Gamma_G,
 *     Gamma_G[i][j] = C(s_i - s_j) - w_i . k_j (members in ascending index
 *     order, xi_G their own stream-1 normals); boxes of one observation keep
 *     phi_i xi_i.  0 (default): every observation on its own.  A box of more
 *     than 32 observations makes condition() return INVALID_ARG; a
 *     non-positive pivot of a box factor returns NOT_POSITIVE_DEFINITE.
 *     Batches and ce_grad_linear use the independent sampling (ce_grad_linear
 *     returns INVALID_ARG while joint sampling is on and some box holds
 *     several observations). */
#define CESIM_PARAM_JOINT_BOXES 8
/*   CESIM_PARAM_SE_CHUNK_NODES (performance and memory only): grid nodes per
 *     chunk of ce_prediction_se, >= 0; 0 (default) takes as many as fit in
 *     16 GiB of work arrays (5 x nodes x stations doubles), at least 64. */
#define CESIM_PARAM_SE_CHUNK_NODES 9
cesim_status ce_set_param(cesim_ctx ctx, int param, int value);

/* ---- launch-shape autotuning ----
 * ce_autotune times the candidate tile shapes of the three draw passes (on
 * the register-FFT path: the largest shape and three successively halved
 * ones, each pass timed on its own with HIP events) and, on the MIXED path
 * after offgrid_nnkrige, the tiles of the grid GEMM (3 only for more than
 * 256 realizations), on
 * min(nreal, 64) realizations written into fields_dev (caller-owned,
 * [nreal][m2][m1]; its contents and the coefficients of the last
 * condition() are overwritten).  The fastest shapes go into a process-wide
 * table keyed by precision and torus size (draw) and by split type,
 * smoothness, grid size, observation count / 512 and realizations rounded
 * up to 256 (GEMM); contexts and batches use table entries unless a
 * parameter above is set.  No result depends on these shapes.  Explicit
 * parameters of ctx are left as they were.  Synchronises. */
cesim_status ce_autotune(cesim_ctx ctx, int nreal, void* fields_dev);

/* The tuning table as JSON lines {"key": "...", "v": [a, b, c]}: save
 * writes every entry; load adds or replaces entries and fails with
 * INVALID_ARG on a line it cannot read or a file it cannot open (entries
 * read before that line are kept). */
cesim_status cesim_tune_save(const char* path);
cesim_status cesim_tune_load(const char* path);
int cesim_tune_entries(void);
void cesim_tune_clear(void);

/* ---- gradient of a linear ensemble statistic ----
 * The adjoint of steps 1-5 of Section 2 (with the local Kriging of
 * Section 2.1 and the Kriging system of eq. (4)) for the statistic
 *   L = (1/R) sum_{r} sum_{g} wgt[g] v_r[g]
 * over the conditional realizations v_r, r = first_real .. first_real +
 * nreal - 1, that ce_simulate(ctx, nreal, seed, first_real) followed by
 * condition(ctx, z, nugget) produces on the FP64 path (noise counters carry
 * the context's CESIM_PARAM_EVENT_ID).  Because every v_r is affine in its
 * noise, L and its derivatives are evaluated once on the mean noises of the
 * R realizations; no field is drawn.  Results (host arrays, caller-owned):
 *   out[0] = L, out[1] = dL/drange, out[2] = dL/dsigma2, out[3] = dL/dnugget,
 *   dz[i]  = dL/dz_i for i < nobs.
 * The range derivative moves the major- and minor-axis ranges together
 * (fixed anisotropy ratio and angle).  wgt_dev: caller-owned device array
 * of m1*m2 doubles, [m2][m1], x fastest; z: host [nobs].  Computes in FP64
 * on either precision (on a MIXED context the draw itself uses FP32 noise,
 * so its ensemble differs from the FP64 one at the 1e-7 level).  Needs
 * offgrid_nnkrige (else BAD_STATE); refactors A when the nugget differs from
 * the last condition().  INVALID_ARG for null pointers, nreal < 1,
 * first_real < 0, a negative or non-finite nugget or a non-finite z, and
 * for nugget = 0 when some observation has gamma_i = 0 (on a grid node;
 * taken as gamma_i <= 1e-12 sigma2, the round-off level of that zero):
 * phi_i = sqrt(nugget + gamma_i) then has an unbounded nugget derivative,
 * so dL/dnugget does not exist; NOT_POSITIVE_DEFINITE when A's Cholesky
 * fails.  Synchronises. */
cesim_status ce_grad_linear(cesim_ctx ctx, const double* z, double nugget, int nreal,
                            uint64_t seed, int first_real, const void* wgt_dev, double* out,
                            double* dz);

/* ---- gradient of any ensemble statistic (vector-Jacobian product) ----
 * For vbar_dev[r][g] (device, nreal x m1*m2 doubles, [r][m2][m1], x
 * fastest, caller-owned) the derivatives of a statistic S with respect to
 * the conditional fields v_r of realizations r = first_real .. first_real
 * + nreal - 1 (the FP64 path, as for ce_grad_linear), returns
 *   out[0] = sum_r vbar[r] . v_r,
 *   out[1..3] = sum_r vbar[r] . dv_r/d(range, sigma2, nugget),
 *   dz[i] = sum_r vbar[r] . dv_r/dz_i,
 * i.e. dS/d(range, sigma2, nugget, z) by the chain rule (the adjoint of
 * steps 1-5 of Section 2 with Section 2.1 and eq. (4)).  Each v_r is affine
 * in its own noise, so the product is the sum of the one-realization linear
 * statistics of ce_grad_linear with weights vbar[r]: cost about nreal times
 * that of one ce_grad_linear call.  Errors and conventions as for
 * ce_grad_linear.  Synchronises. */
cesim_status ce_grad_vjp(cesim_ctx ctx, const double* z, double nugget, int nreal, uint64_t seed,
                         int first_real, const void* vbar_dev, double* out, double* dz);

/* ---- prediction standard errors ----
 * The exact Kriging standard error on the grid (Section 3, eq. (4)),
 *   SE_E(g)^2 = C(0) - K12[g] (K22 + tau^2 I)^{-1} K21[g],
 * and the one the local-Kriging simulation realizes (Section 3.1: the
 * diagonal of (Lambda - I) K11 (Lambda - I)^T + W2 diag(tau^2 + gamma) W2^T,
 * Lambda = W2 W1, W2 = K12 (K22 + tau^2 I)^{-1}), for the stations of the
 * last offgrid_nnkrige and the given nugget (tau^2 >= 0).  Writes m1*m2
 * doubles each ([m2][m1], x fastest) into the caller-owned device arrays
 * se_exact_dev and se_local_dev.  FP64 on either precision; refactors the
 * observation covariance when the nugget differs from the last condition().
 * INVALID_ARG for null pointers or a negative or non-finite nugget, and
 * while joint sampling is on and some box holds several observations (the
 * closed form is that of the independent sampling); BAD_STATE before
 * offgrid_nnkrige, NOT_POSITIVE_DEFINITE when the Cholesky fails.
 * Synchronises. */
cesim_status ce_prediction_se(cesim_ctx ctx, double nugget, void* se_exact_dev,
                              void* se_local_dev);

/* ---- nearest-neighbour Kriging ----
 * The variant of Section 2.2 (variances in Section 3.2): replaces the nobs
 * observations at obs_xy (host, [nobs][2]) with values z (host) by surrogate
 * observations at the grid nodes of their k-node neighbourhoods (the
 * local-Kriging windows of offgrid_nnkrige, k = 4, 16, 36 or 64; overlapping
 * neighbourhoods merged; sites in ascending node index, x fastest).  For the
 * nugget tau^2 >= 0 and A = K22 + tau^2 I, each site j gets the value
 * z_N[j] = K_j2 A^{-1} z and the error variance sigma_N[j]^2 = C(0) -
 * K_j2 A^{-1} K_2j (clamped at 0).  The sites then become the context's
 * stations: each one its own window node, synthetic values y(site) +
 * sqrt(tau^2 + sigma_N^2) xi (xi: the stream-1 normal of the site index), and
 * the observation system K_NN + tau^2 I + diag(sigma_N^2).  Afterwards
 * condition(ctx, z_site, tau^2, fields) draws nearest-neighbour conditional
 * fields and ce_prediction_se(ctx, tau^2, ...) returns the nearest-neighbour
 * standard error SE_N in both maps, both with the same tau^2 as here (the
 * site variances were computed with it); offgrid_nnkrige ends the mode, and
 * ce_grad_linear rejects it (INVALID_ARG).
 * Writes the site count to *nsites, the coordinates to site_xy (host,
 * [capacity][2]) and the values to z_site (host, [capacity]); capacity
 * >= nobs * k always suffices.  INVALID_ARG for null pointers, a bad k, a
 * negative or non-finite nugget or value, more sites than capacity or than
 * 65535; the offgrid_nnkrige statuses for the observations;
 * NOT_POSITIVE_DEFINITE when A is not.  On an error the context holds the
 * observations as after offgrid_nnkrige, or none.  Synchronises. */
cesim_status nn_surrogate(cesim_ctx ctx, int nobs, const double* obs_xy, const double* z,
                          double nugget, int k, int capacity, double* site_xy, double* z_site,
                          int* nsites);

/* ---- batches of independent events ----
 * One event is the whole conditional simulation above (Section 2 with the
 * local Kriging of Section 2.1) for its own covariance, grid, stations,
 * values and realization count.  A batch plans many events once and then
 * runs all of them with one HIP graph launch per call of cesim_batch_run.
 * Event e draws the realizations that a context created with the same
 * covariance, grid and precision, with CESIM_PARAM_EVENT_ID = event_id,
 * would draw with ce_simulate(nreal, seed, first_real + offset) followed by
 * offgrid_nnkrige / condition with the same stations, values and nugget
 * (bit for bit: the same kernels run). */
typedef struct {
  cesim_cov cov;
  cesim_grid grid;            /* t1 = t2 = 0: torus from the ladder */
  int nobs;                   /* >= 1 */
  const double* obs_xy;       /* host [nobs][2]; read during cesim_batch_create only */
  const double* z;            /* host [nobs] observed values; idem */
  double nugget;              /* tau^2 >= 0 */
  int k;                      /* window nodes: 4, 16, 36 or 64 */
  int nreal;                  /* realizations per run, >= 1 */
  int first_real;             /* absolute index of the first realization at offset 0 */
  uint64_t seed;              /* Philox key */
  uint32_t event_id;          /* word 2 of the Philox counter */
  void* fields;               /* device, caller-owned [nreal][m2][m1], double (FP64) or
                                 float (mixed); overwritten by every run */
} cesim_event;

typedef struct cesim_batch_s* cesim_batch;

/* Plans a batch (synchronises hip_stream first): for every event the torus
 * ladder and sqrt(lambda), the local-Kriging set-up and phi; then one
 * grouped FP64 Cholesky of all the K22 + nugget I; then captures the run
 * (per event: CE draw, synthetic observations, the grouped solves of all
 * events, grid GEMM) into one graph.  event_status (nevents entries, may be
 * NULL) receives each event's status (INVALID_ARG, NEGATIVE_EIGENVALUE,
 * OBS_OUTSIDE_GRID, NOT_POSITIVE_DEFINITE, ...); on any failure nothing is
 * kept, *out is NULL and the first failure is returned.  The event table and
 * its host arrays may be freed after the call; the fields buffers must stay
 * allocated until cesim_batch_destroy. */
#define CESIM_BATCH_AUTOTUNE 1   /* flags: run ce_autotune (below) on every event
                                    whose shapes the tuning table lacks, before
                                    the capture (overwrites its fields buffer) */
cesim_status cesim_batch_create(const cesim_event* events, int nevents,
                                cesim_precision prec, void* hip_stream, int flags,
                                cesim_status* event_status, cesim_batch* out);

/* Runs every event of the batch once, asynchronously on the batch's stream,
 * drawing realizations first_real + real_offset .. + nreal - 1 of each event
 * into its fields buffer.  real_offset >= 0.  Calls on one batch are ordered
 * on its stream. */
cesim_status cesim_batch_run(cesim_batch b, int real_offset);

/* Statistics of event e (as ce_get_info); synchronises. */
cesim_status cesim_batch_get_info(cesim_batch b, int e, cesim_info* info);

/* Waits for the batch's runs and releases everything it owns.  NULL is
 * ignored. */
void cesim_batch_destroy(cesim_batch b);

/* create + one run at offset 0 + destroy (returns after the run ended). */
cesim_status cesim_run_events(const cesim_event* events, int nevents,
                              cesim_precision prec, void* hip_stream,
                              cesim_status* event_status);

/* Default timing state of contexts created afterwards (process-wide). */
void cesim_set_default_timing(int enable);

/* Enables (1) or disables (0) stage timing on one context. */
cesim_status ce_set_timing(cesim_ctx ctx, int enable);

/* Accumulated stage times in ms and launch counts (either array may be
 * NULL) for the first nstages stages; synchronises the stream.  reset != 0
 * clears the accumulators after reading. */
cesim_status ce_get_stage_times(cesim_ctx ctx, double* ms, long long* calls,
                                int nstages, int reset);

/* Name of stage i, or "unknown". */
const char* cesim_stage_name(int stage);

/* Device memory freed by destroyed contexts is cached by the library for
 * reuse (so repeated set-ups do not call hipMalloc); this returns the cache
 * to the runtime.  Call only while no context is in use. */
void cesim_release_cached_memory(void);

/* Releases the context and every device buffer it owns (after
 * synchronising its stream).  NULL is ignored. */
void ce_destroy(cesim_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* CESIM_H */
