// abi.hip -- the extern "C" entry points of include/cesim.h: argument
// checks, the torus ladder, context lifetime and host-side test hooks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"

namespace cesim {

// ------------------------------------------------------- caching allocator
namespace {
std::mutex g_cache_mu;
std::multimap<size_t, void*> g_cache;     // size -> block
size_t g_cached_bytes = 0;
constexpr size_t kCacheCap = (size_t)64 << 30;
constexpr size_t kRound = (size_t)2 << 20;
bool g_default_timing = false;
}  // namespace

void* cache_alloc(size_t bytes, size_t* got) {
  bytes = (bytes + kRound - 1) / kRound * kRound;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.lower_bound(bytes);
    if (it != g_cache.end() && it->first <= 2 * bytes) {
      void* p = it->second;
      *got = it->first;
      g_cached_bytes -= it->first;
      g_cache.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    cache_trim();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  *got = bytes;
  return p;
}

void cache_free(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (g_cached_bytes + bytes > kCacheCap) {
    (void)hipFree(p);
    return;
  }
  g_cache.emplace(bytes, p);
  g_cached_bytes += bytes;
}

void cache_trim() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& kv : g_cache) (void)hipFree(kv.second);
  g_cache.clear();
  g_cached_bytes = 0;
}

cesim_status DevBuf::reserve(size_t n) {
  if (n <= bytes && p) return CESIM_OK;
  release();
  size_t got = 0;
  p = cache_alloc(n ? n : 16, &got);
  if (!p) {
    bytes = 0;
    return CESIM_ERR_OUT_OF_MEMORY;
  }
  bytes = got;
  return CESIM_OK;
}

void DevBuf::release() {
  if (p) {
    (void)hipStreamSynchronize(stream);     // work that used the block is done
    cache_free(p, bytes);
  }
  p = nullptr;
  bytes = 0;
}

void DevBuf::release_idle() {
  if (p) cache_free(p, bytes);
  p = nullptr;
  bytes = 0;
}

// ------------------------------------------------------------ stage timer
hipEvent_t StageTimer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

int StageTimer::begin(int stage, hipStream_t s) {
  if (!enabled) return -1;
  hipEvent_t a = get();
  if (!a) return -1;
  (void)hipEventRecord(a, s);
  pending.push_back({stage, a, nullptr});
  return (int)pending.size() - 1;
}

void StageTimer::end(int rec, hipStream_t s) {
  if (rec < 0 || rec >= (int)pending.size()) return;
  hipEvent_t b = get();
  if (!b) return;
  (void)hipEventRecord(b, s);
  pending[rec].b = b;
}

void StageTimer::resolve() {
  for (Rec& r : pending) {
    if (r.b) {
      float ms_ = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms_, r.a, r.b) == hipSuccess) {
        ms[r.stage] += ms_;
        calls[r.stage] += 1;
      }
      pool.push_back(r.b);
    }
    pool.push_back(r.a);
  }
  pending.clear();
}

void StageTimer::destroy() {
  resolve();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

namespace {

bool isfin(double x) { return std::isfinite(x); }

bool smooth(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int next_smooth(int n) {
  n = std::max(n, 1);
  while (!smooth(n)) ++n;
  return n;
}

constexpr int kMaxTorus = 8192;

int nu_code(double nu) {
  if (nu == 0.5) return 0;
  if (nu == 1.0) return 1;
  if (nu == 1.5) return 2;
  return -1;
}

CovDev make_cov(const cesim_cov& c) {
  CovDev d;
  d.nu_code = nu_code(c.nu);
  d.sigma2 = c.sigma2;
  const double cs = std::cos(c.aniso_angle), sn = std::sin(c.aniso_angle);
  const double a = c.aniso_ratio, it = 1.0 / c.range;
  d.theta = c.range;
  if (a == 1.0 && c.aniso_angle == 0.0) {
    d.u00 = it; d.u01 = 0.0; d.u10 = 0.0; d.u11 = it;
  } else {
    d.u00 = cs * it; d.u01 = sn * it; d.u10 = -a * sn * it; d.u11 = a * cs * it;
  }
  return d;
}

cesim_status check_cov(const cesim_cov* c) {
  if (!c) return CESIM_ERR_INVALID_ARG;
  if (nu_code(c->nu) < 0) return CESIM_ERR_INVALID_ARG;
  if (!(isfin(c->sigma2) && c->sigma2 > 0)) return CESIM_ERR_INVALID_ARG;
  if (!(isfin(c->range) && c->range > 0)) return CESIM_ERR_INVALID_ARG;
  if (!(isfin(c->aniso_ratio) && c->aniso_ratio >= 1.0)) return CESIM_ERR_INVALID_ARG;
  if (!isfin(c->aniso_angle)) return CESIM_ERR_INVALID_ARG;
  return CESIM_OK;
}

cesim_status check_grid(const cesim_grid* g) {
  if (!g) return CESIM_ERR_INVALID_ARG;
  if (g->m1 < 2 || g->m2 < 2 || g->m1 > kMaxTorus / 2 || g->m2 > kMaxTorus / 2)
    return CESIM_ERR_INVALID_ARG;
  if (!(isfin(g->x0) && isfin(g->y0) && isfin(g->dx) && isfin(g->dy)))
    return CESIM_ERR_INVALID_ARG;
  if (!(g->dx > 0 && g->dy > 0)) return CESIM_ERR_INVALID_ARG;
  const bool auto_t = g->t1 == 0 && g->t2 == 0;
  if (!auto_t) {
    for (int a = 0; a < 2; ++a) {
      const int t = a ? g->t2 : g->t1, m = a ? g->m2 : g->m1;
      if (t < 2 * m - 1 || t > kMaxTorus || !smooth(t)) return CESIM_ERR_INVALID_ARG;
    }
  }
  return CESIM_OK;
}

}  // namespace
}  // namespace cesim

using namespace cesim;

extern "C" {

const char* cesim_status_string(cesim_status s) {
  switch (s) {
    case CESIM_OK: return "ok";
    case CESIM_ERR_INVALID_ARG: return "invalid argument";
    case CESIM_ERR_NEGATIVE_EIGENVALUE: return "negative circulant eigenvalue (no admissible torus)";
    case CESIM_ERR_NOT_POSITIVE_DEFINITE: return "matrix not positive definite";
    case CESIM_ERR_OBS_OUTSIDE_GRID: return "observation outside the grid";
    case CESIM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case CESIM_ERR_HIP: return "HIP runtime error";
    case CESIM_ERR_BAD_STATE: return "call out of order";
  }
  return "unknown status";
}

static std::vector<DevBuf*> all_bufs(cesim_ctx c) {
  return {&c->tt.tw1_64, &c->tt.tw2_64, &c->tt.tw1_32, &c->tt.tw2_32, &c->s64,
          &c->s32, &c->slb, &c->work, &c->scratch, &c->obs_xy, &c->obs_t32, &c->obs_t64,
          &c->corners, &c->weights, &c->gamma, &c->phi, &c->obs_order, &c->obs_t32s,
          &c->gemm_circ, &c->amat, &c->dinv,
          &c->winv, &c->wtmp, &c->solve_tmp, &c->ainv, &c->ainv_tmp, &c->zdev, &c->coef, &c->coef_b16,
          &c->chat, &c->chat_tmp, &c->yhat, &c->pred_part, &c->pred_next, &c->info_dev, &c->chol_info, &c->winv_seq.dev,
          &c->gwork, &c->gvec, &c->vjp_work, &c->box_of, &c->box_desc, &c->box_members, &c->box_fac,
          &c->sework, &c->nn_extra, &c->nn_work};
}

namespace {
// HIP objects of a context that are slow to create -- the second stream, its
// events and the pinned host words -- kept in a process-wide pool and lent to
// new contexts (all on the device current when they were created).
struct AuxKit {
  hipStream_t aux = nullptr, look = nullptr;
  hipEvent_t ev[7] = {};
  int* info_host = nullptr;
  PinnedStage stage;
};
std::mutex g_kit_mu;
std::vector<AuxKit> g_kits;

void kit_destroy(AuxKit& k) {
  k.stage.release();
  if (k.info_host) (void)hipHostFree(k.info_host);
  for (hipEvent_t e : k.ev)
    if (e) (void)hipEventDestroy(e);
  if (k.aux) (void)hipStreamDestroy(k.aux);
  if (k.look) (void)hipStreamDestroy(k.look);
  k = AuxKit{};
}

// A kit from the pool, or a new one.
cesim_status kit_take(AuxKit& k) {
  {
    std::lock_guard<std::mutex> g(g_kit_mu);
    if (!g_kits.empty()) {
      k = g_kits.back();
      g_kits.pop_back();
      return CESIM_OK;
    }
  }
  bool ok = hipStreamCreateWithFlags(&k.aux, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&k.look, hipStreamNonBlocking) == hipSuccess;
  for (hipEvent_t& e : k.ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&k.info_host, sizeof(int) * 4, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    kit_destroy(k);
    return CESIM_ERR_HIP;
  }
  return CESIM_OK;
}
}  // namespace

void ce_destroy(cesim_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->aux) (void)hipStreamSynchronize(c->aux);
  if (c->look) (void)hipStreamSynchronize(c->look);
  c->timer.destroy();
  for (DevBuf* b : all_bufs(c)) b->release_idle();   // the streams drained above
  AuxKit k;
  k.aux = c->aux;
  k.look = c->look;
  k.ev[0] = c->aux_done;
  k.ev[1] = c->last_use;
  k.ev[2] = c->factor_ready;
  k.ev[3] = c->z_ready;
  k.ev[4] = c->box_ready;
  k.ev[5] = c->la_panel;
  k.ev[6] = c->la_update;
  k.info_host = c->chol_info_host;
  k.stage = c->winv_stage;
  k.stage.pending = false;                 // its copy ran on a drained stream
  bool whole = k.aux && k.look && k.info_host;
  for (hipEvent_t e : k.ev) whole = whole && e;
  if (whole) {
    std::lock_guard<std::mutex> g(g_kit_mu);
    g_kits.push_back(k);
  } else {
    kit_destroy(k);
  }
  delete c;
}

void cesim_release_cached_memory(void) {
  cache_trim();
  std::lock_guard<std::mutex> g(g_kit_mu);
  for (AuxKit& k : g_kits) kit_destroy(k);
  g_kits.clear();
}

void cesim_set_default_timing(int enable) { g_default_timing = enable != 0; }

cesim_status ce_set_param(cesim_ctx c, int param, int value) {
  if (!c) return CESIM_ERR_INVALID_ARG;
  switch (param) {
    case CESIM_PARAM_JOINT_BOXES:
      if (value != 0 && value != 1) return CESIM_ERR_INVALID_ARG;
      c->joint_boxes = value;
      return CESIM_OK;
    case CESIM_PARAM_SE_CHUNK_NODES:
      if (value < 0) return CESIM_ERR_INVALID_ARG;
      c->se_chunk = value;
      return CESIM_OK;
    case CESIM_PARAM_GEMM_TILE:
      if (value < 0 || value > 5) return CESIM_ERR_INVALID_ARG;
      c->gemm_tile = value;
      return CESIM_OK;
    case CESIM_PARAM_DRAW_ROWS:
      if (value < 0 || (value & (value - 1))) return CESIM_ERR_INVALID_ARG;
      c->draw_force.rows = value;
      return CESIM_OK;
    case CESIM_PARAM_DRAW_COLS:
      if (value < 0 || (value & (value - 1))) return CESIM_ERR_INVALID_ARG;
      c->draw_force.lcp = value == 0 ? -1 : __builtin_ctz((unsigned)value);
      return CESIM_OK;
    case CESIM_PARAM_GEMM_SPLIT:
      if (value < 0 || value > 2) return CESIM_ERR_INVALID_ARG;
      c->gemm_split = value;
      return CESIM_OK;
    case CESIM_PARAM_DRAW_CHUNK_PAIRS:
      if (value < 0) return CESIM_ERR_INVALID_ARG;
      c->draw_chunk_pairs = value;
      return CESIM_OK;
    case CESIM_PARAM_EVENT_ID:
      if (value < 0) return CESIM_ERR_INVALID_ARG;
      c->event_id = (uint32_t)value;
      return CESIM_OK;
    default:
      return CESIM_ERR_INVALID_ARG;
  }
}

cesim_status ce_set_timing(cesim_ctx c, int enable) {
  if (!c) return CESIM_ERR_INVALID_ARG;
  c->timer.enabled = enable != 0;
  return CESIM_OK;
}

cesim_status ce_get_stage_times(cesim_ctx c, double* ms, long long* calls, int nstages,
                                int reset) {
  if (!c || nstages < 0 || nstages > ST_COUNT) return CESIM_ERR_INVALID_ARG;
  CESIM_HIP(hipStreamSynchronize(c->stream));
  CESIM_HIP(hipStreamSynchronize(c->aux));
  c->timer.resolve();
  for (int i = 0; i < nstages; ++i) {
    if (ms) ms[i] = c->timer.ms[i];
    if (calls) calls[i] = c->timer.calls[i];
  }
  if (reset) {
    for (int i = 0; i < ST_COUNT; ++i) {
      c->timer.ms[i] = 0;
      c->timer.calls[i] = 0;
    }
  }
  return CESIM_OK;
}

const char* cesim_stage_name(int stage) {
  static const char* names[ST_COUNT] = {
      "setup_torus_base", "setup_fft2_fp64", "setup_eigen_check", "draw_noise_colfft",
      "draw_rowfft_crop", "offgrid_local_krige",
      "obs_cholesky", "synth_obs_rhs", "obs_solve", "coef_split_half", "krige_grid_gemm",
      "krige_predict_fp64", "se_w1k11w1", "se_cov_rows", "se_gemm_xq", "se_reduce"};
  return (stage >= 0 && stage < ST_COUNT) ? names[stage] : "unknown";
}

cesim_status ce_setup(const cesim_cov* cov, const cesim_grid* grid, cesim_precision prec,
                      void* hip_stream, cesim_ctx* out) {
  if (!out) return CESIM_ERR_INVALID_ARG;
  *out = nullptr;
  CESIM_TRY(check_cov(cov));
  CESIM_TRY(check_grid(grid));
  if (prec != CESIM_PREC_FP64 && prec != CESIM_PREC_MIXED) return CESIM_ERR_INVALID_ARG;
  const auto t_start = std::chrono::steady_clock::now();
  cesim_ctx c = new (std::nothrow) cesim_ctx_s();
  if (!c) return CESIM_ERR_OUT_OF_MEMORY;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->cov = *cov;
  c->grid = *grid;
  c->prec = prec;
  c->covd = make_cov(*cov);
  c->gridd = {grid->m1, grid->m2, grid->x0, grid->y0, grid->dx, grid->dy};
  {
    AuxKit k;
    if (kit_take(k) != CESIM_OK) {
      ce_destroy(c);
      return CESIM_ERR_HIP;
    }
    c->aux = k.aux;
    c->aux_done = k.ev[0];
    c->last_use = k.ev[1];
    c->factor_ready = k.ev[2];
    c->z_ready = k.ev[3];
    c->box_ready = k.ev[4];
    c->la_panel = k.ev[5];
    c->la_update = k.ev[6];
    c->look = k.look;
    c->chol_info_host = k.info_host;
    c->winv_stage = k.stage;
  }
  c->chol_info_host[0] = 0;
  for (DevBuf* b : all_bufs(c)) b->stream = c->stream;
  for (DevBuf* b : {&c->amat, &c->dinv, &c->winv, &c->wtmp, &c->zdev, &c->chol_info,
                    &c->winv_seq.dev})
    b->stream = c->aux;                 // written by the work condition() puts on aux
  for (DevBuf* b : {&c->chat, &c->chat_tmp, &c->yhat, &c->pred_part, &c->pred_next})
    b->stream = c->look;                // written by the prediction, on the look-ahead stream
  c->timer.enabled = g_default_timing;
  cesim_status st = CESIM_OK;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess)
      st = CESIM_ERR_HIP;
  }
  if (st == CESIM_OK) st = draw_scratch_address(&c->draw_scratch);
  if (st == CESIM_OK) st = c->info_dev.reserve(sizeof(int) * 4);
  if (st == CESIM_OK) st = c->chol_info.reserve(sizeof(int) * 4);
  if (st == CESIM_OK && hipMemsetAsync(c->chol_info.p, 0, sizeof(int) * 4, c->stream) != hipSuccess)
    st = CESIM_ERR_HIP;
  if (st != CESIM_OK) { ce_destroy(c); return st; }
  std::vector<std::pair<int, int>> cands;
  if (grid->t1 == 0 && grid->t2 == 0) {
    for (int f : {2, 3, 4, 6, 8}) {
      const int a = next_smooth(f * grid->m1), b = next_smooth(f * grid->m2);
      if (a > kMaxTorus || b > kMaxTorus) break;
      if (cands.empty() || cands.back() != std::make_pair(a, b)) cands.push_back({a, b});
    }
  } else {
    cands.push_back({grid->t1, grid->t2});
  }
  bool ok = false;
  for (auto [a, b] : cands) {
    c->torus_tries++;
    bool acc = false;
    st = ce_setup_device(c, a, b, acc);
    if (st != CESIM_OK) { ce_destroy(c); return st; }
    if (acc) {
      c->t1 = a;
      c->t2 = b;
      ok = true;
      break;
    }
  }
  if (!ok) { ce_destroy(c); return CESIM_ERR_NEGATIVE_EIGENVALUE; }
  if (hipStreamSynchronize(c->stream) != hipSuccess) { ce_destroy(c); return CESIM_ERR_HIP; }
  c->ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                          t_start).count();
  *out = c;
  return CESIM_OK;
}

cesim_status ce_simulate(cesim_ctx c, int nreal, uint64_t seed, int first_real, void* fields) {
  if (!c || !fields || nreal < 1 || first_real < 0) return CESIM_ERR_INVALID_ARG;
  if ((long)first_real + nreal > 0x7fffffffL) return CESIM_ERR_INVALID_ARG;
  CESIM_TRY(ce_draw_device(c, nreal, seed, first_real, fields));
  c->have_fields = true;
  c->seed = seed;
  c->first_real = first_real;
  c->nreal = nreal;
  return CESIM_OK;
}

cesim_status ce_simulate_noalloc(cesim_ctx c, int nreal, uint64_t seed, int first_real,
                                 void* fields) {
  if (!c || !fields || nreal < 1 || first_real < 0) return CESIM_ERR_INVALID_ARG;
  if ((long)first_real + nreal > 0x7fffffffL) return CESIM_ERR_INVALID_ARG;
  if (!c->draw_scratch) return CESIM_ERR_BAD_STATE;
  if (draw_pair_bytes(c) > kDrawScratchBytes) return CESIM_ERR_INVALID_ARG;   // one pair must fit
  // same kernels as ce_simulate, pairs in chunks that fit the static array;
  // the stage timer (which records events) is off for the call
  const bool timing = c->timer.enabled;
  c->timer.enabled = false;
  const cesim_status st =
      ce_draw_device(c, nreal, seed, first_real, fields, c->draw_scratch, kDrawScratchBytes);
  c->timer.enabled = timing;
  CESIM_TRY(st);
  c->have_fields = true;
  c->seed = seed;
  c->first_real = first_real;
  c->nreal = nreal;
  return CESIM_OK;
}

// The low 16 bits of v spread to the even bit positions of the result.
static inline uint32_t spread_bits16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// Indices 0..n-1 ordered by key, equal keys in index order (LSD radix sort
// by bytes, skipping the bytes in which all keys agree).
static std::vector<int> stable_radix_order(const std::vector<uint64_t>& key) {
  const int n = (int)key.size();
  std::vector<int> a(n), b(n);
  std::vector<uint64_t> ka(key), kb(n);
  for (int i = 0; i < n; ++i) a[i] = i;
  uint64_t diff = 0;
  for (int i = 1; i < n; ++i) diff |= key[i] ^ key[0];
  for (int sh = 0; sh < 64; sh += 8) {
    if (((diff >> sh) & 0xff) == 0) continue;
    int cnt[257] = {0};
    for (int i = 0; i < n; ++i) ++cnt[((ka[i] >> sh) & 0xff) + 1];
    for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
    for (int i = 0; i < n; ++i) {
      const int dst = cnt[(ka[i] >> sh) & 0xff]++;
      b[dst] = a[i];
      kb[dst] = ka[i];
    }
    a.swap(b);
    ka.swap(kb);
  }
  return a;
}

cesim_status offgrid_nnkrige(cesim_ctx c, int nobs, const double* xy, int k) {
  if (!c || !xy || nobs < 1) return CESIM_ERR_INVALID_ARG;
  int npp = 0;
  switch (k) {
    case 4: npp = 1; break;
    case 16: npp = 2; break;
    case 36: npp = 3; break;
    case 64: npp = 4; break;
    default: return CESIM_ERR_INVALID_ARG;
  }
  const cesim_grid& g = c->grid;
  if (2 * npp > std::min(g.m1, g.m2)) return CESIM_ERR_INVALID_ARG;
  // grid extent with a slack of 1e-12 of its length: (m - 1) dx may round
  // just below the intended edge (for example 1 on the unit square)
  const double ex = (g.m1 - 1) * g.dx, ey = (g.m2 - 1) * g.dy;
  const double xlo = g.x0 - 1e-12 * ex, xhi = g.x0 + ex * (1.0 + 1e-12);
  const double ylo = g.y0 - 1e-12 * ey, yhi = g.y0 + ey * (1.0 + 1e-12);
  for (int i = 0; i < nobs; ++i) {
    const double x = xy[2 * i], y = xy[2 * i + 1];
    if (!(isfin(x) && isfin(y))) return CESIM_ERR_OBS_OUTSIDE_GRID;
    if (x < xlo || x > xhi || y < ylo || y > yhi) return CESIM_ERR_OBS_OUTSIDE_GRID;
  }
  const auto t_start = std::chrono::steady_clock::now();
  CESIM_HIP(hipStreamSynchronize(c->stream));   // host staging below is reused
  CESIM_HIP(hipStreamSynchronize(c->aux));      // buffers below may be reallocated
  c->chol_valid = false;
  c->yhat_valid = false;
  c->nn_active = false;
  c->nobs = 0;
  c->obs_host.assign(xy, xy + 2 * (size_t)nobs);
  CESIM_TRY(c->obs_xy.reserve(sizeof(double) * 2 * nobs));
  CESIM_TRY(c->obs_t64.reserve(sizeof(double2) * nobs));
  CESIM_TRY(c->obs_t32.reserve(sizeof(float2) * nobs));
  CESIM_TRY(c->corners.reserve(sizeof(int2) * nobs));
  CESIM_TRY(c->weights.reserve(sizeof(double) * (size_t)nobs * k));
  CESIM_TRY(c->gamma.reserve(sizeof(double) * nobs));
  CESIM_TRY(c->phi.reserve(sizeof(double) * nobs));
  CESIM_TRY(c->obs_order.reserve(sizeof(int) * nobs));
  const int nchunk = (nobs + kGemmChunk - 1) / kGemmChunk;
  CESIM_TRY(c->obs_t32s.reserve(sizeof(float2) * nobs));
  CESIM_TRY(c->gemm_circ.reserve(sizeof(float4) * nchunk));
  // transformed coordinates: FP64 path U (s - origin); mixed path kappa U (s - origin)
  const CovDev& d = c->covd;
  const double kappa = d.nu_code == 0 ? kLog2e : (d.nu_code == 2 ? kSqrt3 : kSqrt2);
  std::vector<double2> t64(nobs);
  std::vector<float2> t32(nobs);
  // processing order of the gathers: Morton (Z) order of the grid cell
  // (ties in station order); the boxes of several observations (joint
  // sampling) in order of the cell's (column, row), members ascending.
  // Both orders by a stable radix sort of the keys (the station set-up is
  // host time the GPU waits for at every new event).
  std::vector<uint64_t> mkey(nobs), bkey(nobs);
  for (int i = 0; i < nobs; ++i) {
    const double fx = std::floor((xy[2 * i] - g.x0) / g.dx), fy = std::floor((xy[2 * i + 1] - g.y0) / g.dy);
    const uint32_t cx = (uint32_t)std::min(std::max(fx, 0.0), 65535.0);
    const uint32_t cy = (uint32_t)std::min(std::max(fy, 0.0), 65535.0);
    mkey[i] = spread_bits16(cx) | (uint64_t)spread_bits16(cy) << 1;
    // cells start at -1 at the lower slack of the grid's extent
    bkey[i] = (uint64_t)((long)fx + 1) << 32 | (uint64_t)((long)fy + 1);
  }
  const std::vector<int> order = stable_radix_order(mkey);
  const std::vector<int> bord = stable_radix_order(bkey);
  std::vector<int2> box_of(nobs, make_int2(-1, 0));
  std::vector<int4> box_desc;
  std::vector<int> box_members;
  int fac_total = 0, max_box = 0;
  for (int lo = 0; lo < nobs;) {
    int hi = lo + 1;
    while (hi < nobs && bkey[bord[hi]] == bkey[bord[lo]]) ++hi;
    const int sz = hi - lo;
    if (sz > 1) {
      const int d = (int)box_desc.size();
      box_desc.push_back(make_int4((int)box_members.size(), sz, fac_total, 0));
      for (int q = 0; q < sz; ++q) {
        box_members.push_back(bord[lo + q]);
        box_of[bord[lo + q]] = make_int2(d, q);
      }
      fac_total += sz * (sz + 1) / 2;
      max_box = std::max(max_box, sz);
    }
    lo = hi;
  }
  for (int i = 0; i < nobs; ++i) {
    const double hx = xy[2 * i] - g.x0, hy = xy[2 * i + 1] - g.y0;
    const double a = d.u00 * hx + d.u01 * hy, b = d.u10 * hx + d.u11 * hy;
    t64[i] = {a, b};
    t32[i] = {(float)(kappa * a), (float)(kappa * b)};
  }
  // the mixed grid GEMM reads the stations in the same Morton order, in
  // chunks of kGemmChunk: coordinates in that order and the bounding circle
  // of each chunk (centre of its box, radius to the farthest station)
  std::vector<float2> t32s(nobs);
  for (int j = 0; j < nobs; ++j) t32s[j] = t32[order[j]];
  std::vector<float4> circ(nchunk);
  for (int q = 0; q < nchunk; ++q) {
    const int lo = q * kGemmChunk, hi = std::min(nobs, lo + kGemmChunk);
    float xa = t32s[lo].x, xb = xa, ya = t32s[lo].y, yb = ya;
    for (int j = lo + 1; j < hi; ++j) {
      xa = std::min(xa, t32s[j].x); xb = std::max(xb, t32s[j].x);
      ya = std::min(ya, t32s[j].y); yb = std::max(yb, t32s[j].y);
    }
    const float cx = 0.5f * (xa + xb), cy = 0.5f * (ya + yb);
    float r = 0.f;
    for (int j = lo; j < hi; ++j)
      r = std::max(r, std::hypot(t32s[j].x - cx, t32s[j].y - cy));
    circ[q] = make_float4(cx, cy, r, 0.f);
  }
  hipStream_t s = c->stream;
  CESIM_HIP(hipMemcpyAsync(c->obs_t32s.p, t32s.data(), sizeof(float2) * nobs,
                           hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(c->gemm_circ.p, circ.data(), sizeof(float4) * nchunk,
                           hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(c->obs_xy.p, c->obs_host.data(), sizeof(double) * 2 * nobs,
                           hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(c->obs_t64.p, t64.data(), sizeof(double2) * nobs,
                           hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(c->obs_t32.p, t32.data(), sizeof(float2) * nobs,
                           hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(c->obs_order.p, order.data(), sizeof(int) * nobs,
                           hipMemcpyHostToDevice, s));
  CESIM_TRY(c->box_of.reserve(sizeof(int2) * nobs));
  CESIM_TRY(c->box_desc.reserve(sizeof(int4) * std::max<size_t>(1, box_desc.size())));
  CESIM_TRY(c->box_members.reserve(sizeof(int) * std::max<size_t>(1, box_members.size())));
  CESIM_TRY(c->box_fac.reserve(sizeof(double) * std::max(1, fac_total)));
  CESIM_HIP(hipMemcpyAsync(c->box_of.p, box_of.data(), sizeof(int2) * nobs, hipMemcpyHostToDevice,
                           s));
  if (!box_desc.empty()) {
    CESIM_HIP(hipMemcpyAsync(c->box_desc.p, box_desc.data(), sizeof(int4) * box_desc.size(),
                             hipMemcpyHostToDevice, s));
    CESIM_HIP(hipMemcpyAsync(c->box_members.p, box_members.data(),
                             sizeof(int) * box_members.size(), hipMemcpyHostToDevice, s));
  }
  c->nboxes = (int)box_desc.size();
  c->max_box = max_box;
  c->box_fac_valid = false;
  c->nobs = nobs;
  c->k = k;
  c->npp = npp;
  CESIM_TRY(lk_setup_device(c));
  int info[4];
  CESIM_HIP(hipMemcpyAsync(info, c->info_dev.p, sizeof(info), hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));           // also retires the staging vectors
  if (info[0] & 1) {
    c->nobs = 0;
    return CESIM_ERR_NOT_POSITIVE_DEFINITE;
  }
  c->ms_offgrid = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                            t_start).count();
  return CESIM_OK;
}

cesim_status condition(cesim_ctx c, const double* z, double nugget, void* fields) {
  if (!c || !z || !fields) return CESIM_ERR_INVALID_ARG;
  if (c->nobs < 1 || !c->have_fields) return CESIM_ERR_BAD_STATE;
  if (!(isfin(nugget) && nugget >= 0.0)) return CESIM_ERR_INVALID_ARG;
  const int n = c->nobs;
  for (int i = 0; i < n; ++i)
    if (!isfin(z[i])) return CESIM_ERR_INVALID_ARG;
  if (c->z_host_cached.size() != (size_t)n ||
      std::memcmp(c->z_host_cached.data(), z, sizeof(double) * n) != 0) {
    // the upload goes to aux (after the last kernel that read the previous
    // values), so that it does not wait for a draw queued on the stream
    CESIM_HIP(hipStreamSynchronize(c->aux));      // previous upload retired
    c->z_host_cached.assign(z, z + n);
    c->yhat_valid = false;
    CESIM_TRY(c->zdev.reserve(sizeof(double) * n));
    CESIM_TRY(aux_wait_last_use(c));
    CESIM_HIP(hipMemcpyAsync(c->zdev.p, c->z_host_cached.data(), sizeof(double) * n,
                             hipMemcpyHostToDevice, c->aux));
    CESIM_HIP(hipEventRecord(c->z_ready, c->aux));
    c->z_pending = true;
    c->aux_pending = true;
  }
  const cesim_status st = condition_device(c, nugget, fields);
  // the batch is conditional now: conditioning it again would add the
  // Kriging correction twice, so a further condition() needs a new draw
  if (st == CESIM_OK) c->have_fields = false;
  return st;
}

cesim_status ce_get_info(cesim_ctx c, cesim_info* info) {
  if (!c || !info) return CESIM_ERR_INVALID_ARG;
  CESIM_HIP(hipStreamSynchronize(c->stream));
  cesim_info r{};
  r.t1 = c->t1;
  r.t2 = c->t2;
  r.lam_min = c->lam_min;
  r.lam_max = c->lam_max;
  r.lam_sum = c->lam_sum;
  r.max_imag = c->max_imag;
  r.nobs = c->nobs;
  r.k = c->k;
  r.ms_setup = c->ms_setup;
  r.ms_offgrid = c->ms_offgrid;
  r.precision = (int)c->prec;
  r.torus_tries = c->torus_tries;
  if (c->nobs > 0) {
    std::vector<double> gm(c->nobs);
    CESIM_HIP(hipMemcpy(gm.data(), c->gamma.p, sizeof(double) * c->nobs, hipMemcpyDeviceToHost));
    r.gamma_min = *std::min_element(gm.begin(), gm.end());
    r.gamma_max = *std::max_element(gm.begin(), gm.end());
  }
  *info = r;
  return CESIM_OK;
}

cesim_status ce_copy_spectrum(cesim_ctx c, double* dev_out) {
  if (!c || !dev_out) return CESIM_ERR_INVALID_ARG;
  CESIM_HIP(hipMemcpyAsync(dev_out, c->s64.p, sizeof(double) * (size_t)c->t1 * c->t2,
                           hipMemcpyDeviceToDevice, c->stream));
  return CESIM_OK;
}

cesim_status offgrid_copy_weights(cesim_ctx c, int* corners, double* w, double* gam) {
  if (!c) return CESIM_ERR_INVALID_ARG;
  if (c->nobs < 1) return CESIM_ERR_BAD_STATE;
  const size_t n = c->nobs;
  if (corners)
    CESIM_HIP(hipMemcpyAsync(corners, c->corners.p, sizeof(int2) * n, hipMemcpyDeviceToDevice,
                             c->stream));
  if (w)
    CESIM_HIP(hipMemcpyAsync(w, c->weights.p, sizeof(double) * n * c->k,
                             hipMemcpyDeviceToDevice, c->stream));
  if (gam)
    CESIM_HIP(hipMemcpyAsync(gam, c->gamma.p, sizeof(double) * n, hipMemcpyDeviceToDevice,
                             c->stream));
  return CESIM_OK;
}

cesim_status condition_copy_coefficients(cesim_ctx c, double* dev_out) {
  if (!c || !dev_out) return CESIM_ERR_INVALID_ARG;
  if (c->nobs < 1 || !c->coef.p) return CESIM_ERR_BAD_STATE;
  return copy_coefficients_device(c, dev_out);
}

cesim_status cesim_covariance_host(const cesim_cov* cov, int n, const double* hx,
                                   const double* hy, double* out) {
  CESIM_TRY(check_cov(cov));
  if (n < 0 || (n > 0 && (!hx || !hy || !out))) return CESIM_ERR_INVALID_ARG;
  const CovDev d = make_cov(*cov);
  for (int i = 0; i < n; ++i) out[i] = cov_eval(d, hx[i], hy[i]);
  return CESIM_OK;
}

cesim_status cesim_philox_host(uint64_t seed, int n, const uint32_t* ctr0, uint32_t c1,
                               uint32_t c2, uint32_t c3, uint32_t* out) {
  if (n < 0 || (n > 0 && (!ctr0 || !out))) return CESIM_ERR_INVALID_ARG;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  for (int i = 0; i < n; ++i) {
    const u32x4 w = philox4x32_10({ctr0[i], c1, c2, c3}, k0, k1);
    out[4 * i] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
  }
  return CESIM_OK;
}

}  // extern "C"
