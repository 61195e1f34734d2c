// batch.hip -- many independent events (each one the conditional simulation
// of Section 2 with the local Kriging of Section 2.1, with its own
// covariance, grid, stations, values and realization count), planned once
// and then run as one HIP graph launch per batch of realizations.
//
// Plan (cesim_batch_create, synchronising):
//   per event: torus ladder and sqrt(lambda) (the ladder is a host decision),
//   local-Kriging setup, upload of the observed values, phi = sqrt(tau^2 +
//   gamma); then one grouped blocked Cholesky over all events (step kb
//   factors diagonal block kb of every system at once); buffers for every
//   later step are reserved here; optionally the launch shapes of shapes not
//   yet in the tuning table are tuned.
// Run (cesim_batch_run, asynchronous): one graph holding, for every event,
//   the CE draw, the synthetic observations and right-hand sides, the
//   grouped forward / backward solves of all events, and the grid GEMM.
//   The realization offset is read by the noise kernels from device memory,
//   so replays draw later realizations without re-capturing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

using namespace cesim;

struct cesim_batch_s {
  hipStream_t user = nullptr;         // caller's stream: runs are ordered on it
  hipStream_t own = nullptr;          // private stream for planning and capture
  cesim_precision prec = CESIM_PREC_FP64;
  std::vector<cesim_ctx> ctx;
  std::vector<cesim_event> ev;        // copies; host pointers are not kept
  DevBuf work;                        // pair buffers of the draw, shared by all events
  DevBuf roff;                        // realization offset of the current run (int)
  GroupedSeq solve;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double ms_plan = 0;
};

namespace {

__global__ void k_set_int(int* p, int v) { *p = v; }

cesim_status check_event(const cesim_event& e) {
  if (e.nobs < 1 || !e.obs_xy || !e.z || !e.fields || e.nreal < 1 || e.first_real < 0)
    return CESIM_ERR_INVALID_ARG;
  if ((long)e.first_real + e.nreal > INT_MAX) return CESIM_ERR_INVALID_ARG;
  if (!(std::isfinite(e.nugget) && e.nugget >= 0.0)) return CESIM_ERR_INVALID_ARG;
  for (int i = 0; i < e.nobs; ++i)
    if (!std::isfinite(e.z[i])) return CESIM_ERR_INVALID_ARG;
  return CESIM_OK;
}

void destroy_batch(cesim_batch b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->user);
  if (b->own) (void)hipStreamSynchronize(b->own);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (cesim_ctx c : b->ctx)
    if (c) {
      c->ext_work = nullptr;
      c->roff = nullptr;
      ce_destroy(c);
    }
  b->solve.dev.release();
  b->work.release();
  b->roff.release();
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
}

// Steady-state work of every event, on b->own (under capture).
cesim_status record_run(cesim_batch b) {
  for (size_t e = 0; e < b->ctx.size(); ++e) {
    cesim_ctx c = b->ctx[e];
    const cesim_event& ev = b->ev[e];
    CESIM_TRY(ce_draw_device(c, ev.nreal, ev.seed, ev.first_real, ev.fields));
  }
  for (size_t e = 0; e < b->ctx.size(); ++e)
    CESIM_TRY(lk_synth_rhs_device(b->ctx[e], b->ev[e].fields, b->ctx[e]->coef.as<double>(),
                                  b->prec == CESIM_PREC_FP64));
  CESIM_TRY(b->solve.launch(b->own));
  for (size_t e = 0; e < b->ctx.size(); ++e)
    CESIM_TRY(krige_grid_device(b->ctx[e], b->ctx[e]->coef.as<double>(), b->ev[e].fields));
  return CESIM_OK;
}

cesim_status plan(cesim_batch b, cesim_status* status, int flags) {
  const int ne = (int)b->ev.size();
  std::vector<double> tau2(ne);
  // per-event set-up: ladder, local Kriging, values, phi
  for (int e = 0; e < ne; ++e) {
    const cesim_event& ev = b->ev[e];
    cesim_ctx c = nullptr;
    cesim_status st = ce_setup(&ev.cov, &ev.grid, b->prec, b->own, &c);
    if (st == CESIM_OK) {
      b->ctx[e] = c;
      c->timer.enabled = false;
      st = offgrid_nnkrige(c, ev.nobs, ev.obs_xy, ev.k);
    }
    if (st == CESIM_OK) {
      c->z_host_cached.assign(ev.z, ev.z + ev.nobs);
      st = c->zdev.reserve(sizeof(double) * ev.nobs);
      if (st == CESIM_OK &&
          hipMemcpyAsync(c->zdev.p, c->z_host_cached.data(), sizeof(double) * ev.nobs,
                         hipMemcpyHostToDevice, b->own) != hipSuccess)
        st = CESIM_ERR_HIP;
    }
    if (st == CESIM_OK) st = lk_phi_device(c, ev.nugget);
    if (st == CESIM_OK) st = krige_reserve(c, ev.nreal);
    if (status) status[e] = st;
    if (st != CESIM_OK) return st;
    tau2[e] = ev.nugget;
    c->event_id = ev.event_id;
  }
  // one grouped Cholesky over all events
  std::vector<int> not_pd;
  CESIM_TRY(chol_factor_batch(b->ctx, tau2, b->own, not_pd));
  cesim_status first = CESIM_OK;
  for (int e = 0; e < ne; ++e)
    if (not_pd[e]) {
      if (status) status[e] = CESIM_ERR_NOT_POSITIVE_DEFINITE;
      if (first == CESIM_OK) first = CESIM_ERR_NOT_POSITIVE_DEFINITE;
    }
  if (first != CESIM_OK) return first;
  // realization offset (the draw sizes its pairs for offsets of either
  // parity), shared pair buffers, solve launches
  CESIM_TRY(b->roff.reserve(sizeof(int)));
  for (int e = 0; e < ne; ++e) b->ctx[e]->roff = b->roff.as<int>();
  size_t wbytes = 0;
  for (int e = 0; e < ne; ++e)
    wbytes = std::max(wbytes, draw_pair_bytes(b->ctx[e]) *
                                  (size_t)draw_chunk_pairs(b->ctx[e], b->ev[e].nreal,
                                                           b->ev[e].first_real));
  CESIM_TRY(b->work.reserve(wbytes));
  k_set_int<<<1, 1, 0, b->own>>>(b->roff.as<int>(), 0);
  CESIM_HIP(hipGetLastError());
  std::vector<double*> X(ne);
  std::vector<int> R(ne);
  for (int e = 0; e < ne; ++e) {
    cesim_ctx c = b->ctx[e];
    const cesim_event& ev = b->ev[e];
    X[e] = c->coef.as<double>();
    R[e] = ev.nreal;
    c->ext_work = b->work.p;
    c->ext_work_bytes = b->work.bytes;
    c->roff = b->roff.as<int>();
    c->stream = b->own;
    c->have_fields = true;
    c->seed = ev.seed;
    c->first_real = ev.first_real;
    c->nreal = ev.nreal;
  }
  if (b->prec == CESIM_PREC_MIXED)
    for (int e = 0; e < ne; ++e) CESIM_TRY(predict_device(b->ctx[e], b->own));
  if (flags & CESIM_BATCH_AUTOTUNE)
    for (int e = 0; e < ne; ++e)
      if (!tune_has_entries(b->ctx[e], b->ev[e].nreal))
        CESIM_TRY(ce_autotune(b->ctx[e], b->ev[e].nreal, b->ev[e].fields));
  CESIM_TRY(chol_solve_batch_plan(b->ctx, X, R, b->solve));
  CESIM_TRY(b->solve.upload(b->own));
  // capture the run
  CESIM_HIP(hipStreamBeginCapture(b->own, hipStreamCaptureModeRelaxed));
  const cesim_status rec = record_run(b);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->own, &g);
  if (rec != CESIM_OK || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rec != CESIM_OK ? rec : CESIM_ERR_HIP;
  }
  b->graph = g;
  CESIM_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  CESIM_HIP(hipStreamSynchronize(b->own));
  return CESIM_OK;
}

}  // namespace

extern "C" {

cesim_status cesim_batch_create(const cesim_event* events, int nevents, cesim_precision prec,
                                void* hip_stream, int flags, cesim_status* event_status,
                                cesim_batch* out) {
  if (!out) return CESIM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!events || nevents < 1 || (flags & ~CESIM_BATCH_AUTOTUNE)) return CESIM_ERR_INVALID_ARG;
  if (prec != CESIM_PREC_FP64 && prec != CESIM_PREC_MIXED) return CESIM_ERR_INVALID_ARG;
  cesim_status first = CESIM_OK;
  for (int e = 0; e < nevents; ++e) {
    const cesim_status st = check_event(events[e]);
    if (event_status) event_status[e] = st;
    if (st != CESIM_OK && first == CESIM_OK) first = st;
  }
  if (first != CESIM_OK) return first;
  const auto t0 = std::chrono::steady_clock::now();
  cesim_batch b = new (std::nothrow) cesim_batch_s();
  if (!b) return CESIM_ERR_OUT_OF_MEMORY;
  b->user = static_cast<hipStream_t>(hip_stream);
  b->prec = prec;
  b->ev.assign(events, events + nevents);
  b->ctx.assign(nevents, nullptr);
  if (hipStreamSynchronize(b->user) != hipSuccess ||
      hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess) {
    destroy_batch(b);
    return CESIM_ERR_HIP;
  }
  b->work.stream = b->roff.stream = b->solve.dev.stream = b->own;
  const cesim_status st = plan(b, event_status, flags);
  for (auto& ev : b->ev) {
    ev.obs_xy = nullptr;
    ev.z = nullptr;
  }
  if (st != CESIM_OK) {
    destroy_batch(b);
    return st;
  }
  b->ms_plan = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                   .count();
  *out = b;
  return CESIM_OK;
}

cesim_status cesim_batch_run(cesim_batch b, int real_offset) {
  if (!b || !b->exec || real_offset < 0) return CESIM_ERR_INVALID_ARG;
  for (const cesim_event& ev : b->ev)
    if ((long)ev.first_real + real_offset + ev.nreal > INT_MAX) return CESIM_ERR_INVALID_ARG;
  k_set_int<<<1, 1, 0, b->user>>>(b->roff.as<int>(), real_offset);
  CESIM_HIP(hipGetLastError());
  CESIM_HIP(hipGraphLaunch(b->exec, b->user));
  return CESIM_OK;
}

cesim_status cesim_batch_get_info(cesim_batch b, int e, cesim_info* info) {
  if (!b || !info || e < 0 || e >= (int)b->ctx.size()) return CESIM_ERR_INVALID_ARG;
  CESIM_HIP(hipStreamSynchronize(b->user));
  return ce_get_info(b->ctx[e], info);
}

void cesim_batch_destroy(cesim_batch b) { destroy_batch(b); }

cesim_status cesim_run_events(const cesim_event* events, int nevents, cesim_precision prec,
                              void* hip_stream, cesim_status* event_status) {
  cesim_batch b = nullptr;
  CESIM_TRY(cesim_batch_create(events, nevents, prec, hip_stream, 0, event_status, &b));
  const cesim_status st = cesim_batch_run(b, 0);
  destroy_batch(b);              // synchronises the stream first
  return st;
}

}  // extern "C"
