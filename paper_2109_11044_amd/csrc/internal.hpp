// internal.hpp -- context and host-side plumbing shared by the library's
// translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/cesim.h"
#include "devmath.hpp"
#include "fft.hpp"

namespace cesim {

#define CESIM_HIP(call)                                     \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return CESIM_ERR_HIP;             \
  } while (0)

#define CESIM_TRY(call)                                     \
  do {                                                      \
    cesim_status s_ = (call);                               \
    if (s_ != CESIM_OK) return s_;                          \
  } while (0)

// Grid in device form.
struct GridDev {
  int m1, m2;
  double x0, y0, dx, dy;
};

// Process-wide caching allocator: freed blocks are kept for reuse so that
// repeated set-ups do not call hipMalloc / hipFree (which synchronise the
// device).  A block is handed back only after the stream that used it has
// drained.
void* cache_alloc(size_t bytes, size_t* got);
void cache_free(void* p, size_t bytes);
void cache_trim();

// A device allocation owned by the context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;     // stream whose work last used the block
  cesim_status reserve(size_t n);   // grows, never shrinks; contents lost
  void release();
  void release_idle();              // no work that uses the block is pending
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Width of the diagonal blocks of the observation factor whose inverses
// (winv) the blocked substitutions apply.
constexpr int kSolveBlock = 256;

// Observations per k-chunk of the mixed grid GEMM.
constexpr int kGemmChunk = 32;

// Stages timed with HIP events when timing is enabled on a context.
enum Stage {
  ST_SETUP_BASE = 0, ST_SETUP_FFT, ST_SETUP_EIG, ST_DRAW_PASS_A, ST_DRAW_PASS_B,
  ST_LK_SETUP, ST_CHOL, ST_SYNTH_RHS, ST_SOLVE, ST_COEF_SPLIT, ST_KRIGE_GEMM, ST_PREDICT,
  ST_SE_Q, ST_SE_COV_ROWS, ST_SE_GEMM, ST_SE_REDUCE,
  ST_COUNT
};

struct StageTimer {
  bool enabled = false;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double ms[ST_COUNT] = {0};
  long calls[ST_COUNT] = {0};
  hipEvent_t get();
  int begin(int stage, hipStream_t s);      // returns a record index or -1
  void end(int rec, hipStream_t s);
  void resolve();                           // after a stream synchronise
  void destroy();
};

// FP64 GEMM C = alpha A B + beta C with element strides A(i,k) = A[i sai + k sak],
// B(k,j) = B[k sbk + j sbj], C(i,j) = C[i sci + j scj].
struct GemmArgs {
  int M, N, K;
  double alpha, beta;
  const double* A; long sai, sak;
  const double* B; long sbk, sbj;
  double* C; long sci, scj;
};

// One 64 x 64 diagonal block of a blocked Cholesky factorisation.
struct DiagDesc {
  double* A;        // n x n, row-major, factored in place (lower)
  int n, k0, nbk;
  double* dinv;     // 64 x 64 inverse of the block's factor
  int* info;        // bit 2 set on a non-positive pivot
};

// A recorded sequence of grouped launches over several independent systems
// (diagonal factorisations and FP64 GEMMs), uploaded once and then launched
// any number of times without host work beyond the launches themselves.
// Pinned host staging of an asynchronous upload: the host copy stays
// untouched until the copy recorded by `done` has run.
struct PinnedStage {
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  cesim_status acquire(size_t n);   // waits for the previous copy; grows to n bytes
  cesim_status mark(hipStream_t s); // records done after a copy queued on s
  void release();
};

struct GroupedSeq {
  struct Launch { int kind, first, count, blocks, pfx; };   // kind: 0 diag, 1 GEMM, 2 lower GEMM
  std::vector<DiagDesc> diag;
  std::vector<GemmArgs> gemm;
  std::vector<int> pfx;
  std::vector<Launch> launches;
  DevBuf dev;
  DiagDesc* d_diag = nullptr;
  GemmArgs* d_gemm = nullptr;
  int* d_pfx = nullptr;
  void add_diag(const std::vector<DiagDesc>& v);
  void add_gemm(const std::vector<GemmArgs>& v, bool lower);   // empty problems are dropped
  void clear();                                                // keeps the device buffer
  cesim_status upload(hipStream_t s);                          // synchronises s
  cesim_status upload_async(hipStream_t s, PinnedStage& st);   // does not synchronise
  cesim_status launch(hipStream_t s) const;
};

// Tile shape of the register-FFT draw passes: log2 of the columns per
// workgroup of pass A (-1: largest) and the rows per workgroup of pass B
// (0: largest).  Results do not depend on it.
struct DrawShape {
  int lcp = -1, rows = 0;
};

struct TorusTables {
  Plan p1, p2;                      // plans along x (t1) and y (t2)
  DevBuf tw1_64, tw2_64, tw1_32, tw2_32;   // twiddles exp(-2 pi i t / T)
};

}  // namespace cesim

struct cesim_ctx_s {
  hipStream_t stream = nullptr;
  // condition() runs the observation factorisation, the upload of the
  // observed values and the FP64 prediction -- which do not need the drawn
  // fields -- on aux, overlapping the draw queued on stream.  aux first waits
  // for last_use (recorded on stream after the previous condition()'s last
  // kernel); stream waits for aux_done before it uses their results.
  // factor_ready: the factor and block inverses are complete (the solves
  // may start); z_ready: the observed values are on the device.
  hipStream_t aux = nullptr;
  hipEvent_t aux_done = nullptr, last_use = nullptr, factor_ready = nullptr, z_ready = nullptr;
  hipEvent_t box_ready = nullptr;   // box factors of the joint sampling are complete
  // Look-ahead of the factorization: the trailing updates beyond the next
  // block column run on `look` while the next diagonal block is factored;
  // la_panel: a panel and its next-column update are done; la_update: the
  // look stream's trailing update is done.
  hipStream_t look = nullptr;
  hipEvent_t la_panel = nullptr, la_update = nullptr;
  bool last_use_valid = false, aux_pending = false, z_pending = false;
  cesim_cov cov{};
  cesim_grid grid{};
  cesim_precision prec = CESIM_PREC_FP64;
  cesim::CovDev covd{};
  cesim::GridDev gridd{};
  int t1 = 0, t2 = 0;
  int num_cu = 0;                   // compute units of the device the context runs on
  double lam_min = 0, lam_max = 0, lam_sum = 0, max_imag = 0;
  int torus_tries = 0;
  double ms_setup = 0, ms_offgrid = 0;

  cesim::TorusTables tt;
  cesim::StageTimer timer;
  cesim::DevBuf s64, s32;           // sqrt(lambda) / (t1 t2), [t2][t1]
  // the same for the register draw path, in its precision and blocked by 8
  // columns, [t1 / 8][t2][8], so that the column pass reads it contiguously
  cesim::DevBuf slb;
  cesim::DevBuf work;               // pair buffers of the draw / setup FFT
  cesim::DevBuf scratch;            // small reductions

  // local Kriging
  int nobs = 0, k = 0, npp = 0;
  cesim::DevBuf obs_xy;             // [n][2] FP64
  cesim::DevBuf obs_t32;            // [n] float2: transformed coordinates (mixed)
  cesim::DevBuf obs_t64;            // [n] double2: transformed coordinates (FP64)
  cesim::DevBuf corners, weights, gamma, phi;
  cesim::DevBuf obs_order;          // [n] int: observations in Morton order of their grid cell
  // the mixed grid GEMM's station order (the same Morton order) and, per
  // chunk of kGemmChunk stations in it, a bounding circle (centre, radius)
  // in the GEMM's scaled coordinates
  cesim::DevBuf obs_t32s;           // [n] float2: transformed coordinates in that order
  cesim::DevBuf gemm_circ;          // [ceil(n / kGemmChunk)] float4
  // boxes holding several observations (joint sampling, CESIM_PARAM_JOINT_BOXES)
  int joint_boxes = 0;              // switched on by the parameter
  int se_chunk = 0;                 // grid nodes per standard-error chunk (0: auto)
  // nearest-neighbour Kriging: the stations are surrogate grid sites whose
  // nugget is tau^2 + nn_extra[i] (set by nn_surrogate, cleared by offgrid_nnkrige)
  bool nn_active = false;
  cesim::DevBuf nn_extra;
  cesim::DevBuf nn_work;
  int nboxes = 0, max_box = 0;      // boxes of several observations; largest size
  bool box_fac_valid = false;       // box_fac matches the stations and chol_nugget
  cesim::DevBuf box_of;             // [n] int2: {box, row in box} or {-1, 0}
  cesim::DevBuf box_desc;           // [nboxes] int4: {first member, size, factor offset, 0}
  cesim::DevBuf box_members;        // observation indices of each box, ascending
  cesim::DevBuf box_fac;            // packed lower factors of tau^2 I + Gamma_G
  double gamma_min = 0, gamma_max = 0;
  std::vector<double> obs_host;

  // conditioning
  bool chol_valid = false;
  bool yhat_valid = false;          // mixed path: chat and yhat match the factor and z
  double chol_nugget = -1.0;
  cesim::DevBuf amat;               // n x n: K22 + tau^2 I, then its Cholesky factor
  cesim::DevBuf dinv;               // inverses of the 64 x 64 diagonal blocks
  cesim::DevBuf winv;               // inverses of the kSolveBlock-wide diagonal blocks
  cesim::DevBuf wtmp;               // products formed while building winv
  cesim::DevBuf solve_tmp;          // [R][n]: second buffer of the substitutions
  bool ainv_valid = false;          // ainv holds A^{-1} of the current factor
  cesim::DevBuf ainv;               // n x n FP64 A^{-1} (mixed path, repeated calls)
  cesim::DevBuf ainv_tmp;           // second buffer while it is formed
  cesim::DevBuf zdev;               // observed values
  cesim::DevBuf coef;               // [R][n] FP64: z - z*, then the coefficients
  cesim::DevBuf coef_b16;           // half-precision hi / lo coefficients + column scales (mixed)
  cesim::DevBuf chat;               // mixed path: A^{-1} z, FP64 [n]
  cesim::DevBuf chat_tmp;           // second buffer of that solve
  cesim::DevBuf yhat;               // mixed path: K12 A^{-1} z on the grid, FP32 [M]
  cesim::DevBuf pred_part;          // its partial sums per slice of stations, FP64 [S][M]
  cesim::DevBuf pred_next;          // item counter of the prediction kernel
  cesim::DevBuf info_dev;           // int flags of the local-Kriging setup
  cesim::DevBuf chol_info;          // int[4]: bit 2 of [0] marks a failed factorisation;
                                    // the grid GEMM leaves the fields alone when it is set
  int* chol_info_host = nullptr;    // pinned copy, valid once factor_ready has completed
  cesim::DevBuf gwork;              // gradient: one FP64 pair buffer + d sqrt(lambda)
  cesim::DevBuf gvec;               // gradient: mean noises, fields and vectors
  cesim::DevBuf vjp_work;           // vector-Jacobian product: per-realization arrays
  cesim::DevBuf sework;             // standard errors: chunk arrays and W1 K11 W1^T
  cesim::GroupedSeq winv_seq;       // launches that build winv (kept until they have run)
  cesim::PinnedStage winv_stage;
  std::vector<double> z_host_cached;

  int gemm_tile = 0;                // mixed grid GEMM tile, 1-5 (0: tuning table, else 1)
  cesim::DrawShape draw_force;      // tile shape set with ce_set_param (wins over the table)
  int gemm_split = 0;               // 0: FP16 x3, 1: BF16 x3
  int draw_chunk_pairs = 0;         // pairs per draw launch (0: by a 2 GiB budget)

  // batched runs: Philox event word, device realization offset, lent pair buffers
  uint32_t event_id = 0;
  const int* roff = nullptr;
  void* ext_work = nullptr;
  size_t ext_work_bytes = 0;
  // device address of this device's static pair-buffer array (the draw of
  // ce_simulate_noalloc), looked up at set-up
  void* draw_scratch = nullptr;

  // last simulate
  bool have_fields = false;
  uint64_t seed = 0;
  int first_real = 0, nreal = 0;
};

namespace cesim {

// Kernels launched from the ABI layer (defined in the .hip files).
cesim_status ce_setup_device(cesim_ctx c, int t1, int t2, bool& accepted);
// work / work_bytes: pair buffers lent by the caller (nullptr: the
// context's own, or a batch's).
cesim_status ce_draw_device(cesim_ctx c, int nreal, uint64_t seed, int first_real, void* fields,
                            void* work = nullptr, size_t work_bytes = 0);
cesim_status lk_setup_device(cesim_ctx c);
cesim_status condition_device(cesim_ctx c, double nugget, void* fields);
cesim_status lk_phi_device(cesim_ctx c, double tau2);
cesim_status lk_synth_rhs_device(cesim_ctx c, const void* fields, double* rhs, bool with_z);
cesim_status predict_device(cesim_ctx c, hipStream_t s);
cesim_status chol_factor_device(cesim_ctx c, double tau2, hipStream_t s, bool clear_info = true);
cesim_status box_factor_device(cesim_ctx c, double tau2, hipStream_t s);
bool joint_active(cesim_ctx c);
constexpr int kMaxJointBox = 32;   // observations per box of the joint sampling
cesim_status ce_grad_fields_device(cesim_ctx c, const double2* zeta_bar, double* yb, double* dyb);
cesim_status grad_dsqrt_device(cesim_ctx c, double* ds, double2* tmp);
cesim_status draw_f64_spectrum_device(cesim_ctx c, int nreal, uint64_t seed, int first_real,
                                      double* fields, const double* sl, double* slb);
// rows_in_place: C is A's storage with N <= 64 (a workgroup must read the
// whole row block before writing it), which keeps 64 x 64 tiles.
cesim_status gemm_f64(const GemmArgs& g, bool lower, hipStream_t s, bool rows_in_place = false);
// R sets (fields [R][M], noises [R][n], outputs [R][4n]); R = 1: one set.
cesim_status lk_grad_device(cesim_ctx c, double tau2, const double* yb, const double* dyb,
                            const double* xib, double* out, int R = 1);
// identity: X holds I (R = n) and Y zeros; the forward steps skip the rows
// whose forward solution is still zero.
cesim_status chol_solve_device(cesim_ctx c, double* X, int R, hipStream_t s, double* Y,
                               int stage = ST_SOLVE, bool identity = false);
cesim_status chol_solve_vec_device(cesim_ctx c, const double* b, double* x, hipStream_t s,
                                   double* y, int stage);
// Repeated mixed-path calls of at most kInverseMaxReal realizations on one
// factor of at most kInverseMaxObs stations use A^{-1}.
constexpr int kInverseMaxObs = 8192;
constexpr int kInverseMaxReal = 128;
cesim_status inverse_device(cesim_ctx c, hipStream_t s);
cesim_status apply_inverse_device(cesim_ctx c, const double* X, int R, double* Y, hipStream_t s);
cesim_status aux_wait_last_use(cesim_ctx c);
cesim_status copy_coefficients_device(cesim_ctx c, double* out);
cesim_status krige_grid_device(cesim_ctx c, const double* X, void* fields);
cesim_status krige_reserve(cesim_ctx c, int R);
cesim_status chol_factor_batch(const std::vector<cesim_ctx>& cs, const std::vector<double>& tau2,
                               hipStream_t s, std::vector<int>& not_pd);
cesim_status chol_solve_batch_plan(const std::vector<cesim_ctx>& cs,
                                   const std::vector<double*>& X, const std::vector<int>& R,
                                   GroupedSeq& seq);
cesim_status make_plan(int T, Plan& p);
size_t draw_pair_bytes(cesim_ctx c);
// Launch shapes in force: explicit settings, else the tuning table, else
// the largest shapes / one node fragment.
DrawShape draw_shape(cesim_ctx c);
int gemm_tile(cesim_ctx c, int R);
bool register_draw_path(cesim_ctx c);
bool register_draw_torus(int t1, int t2);
DrawShape draw_shape_limits(cesim_ctx c);   // largest shapes of the register path
bool tune_has_entries(cesim_ctx c, int R);  // table holds this context's shapes
int draw_npairs(cesim_ctx c, int nreal, int first_real);
int draw_chunk_pairs(cesim_ctx c, int nreal, int first_real);
cesim_status make_twiddles(int T, DevBuf& tw64, DevBuf& tw32, hipStream_t s);
// Size of the static pair-buffer array of ce_simulate_noalloc (one per
// device) and the current device's address of it.
constexpr size_t kDrawScratchBytes = (size_t)64 << 20;
cesim_status draw_scratch_address(void** out);

}  // namespace cesim
