// tune.hip -- launch-shape autotuning.
//
// Tunable: the tile shapes of the two register-FFT draw passes (columns per
// workgroup of the column pass A, rows per workgroup of the row pass B)
// and the workgroup tile of the mixed grid GEMM.  None of them
// changes a single bit of any result (each output element sees the same
// operations in the same order), so tuning affects speed only.  The radix
// sequence of the transforms is fixed by design and not tuned.
//
// Chosen shapes live in a process-wide table keyed by problem shape:
//   "drawAB p<precision> <t1>x<t2>"               -> log2 cols (A), rows (B), 0
//   "gemm s<split> nu<code> M<nodes> n<n/512> R<Rp>" -> GEMM tile
// and can be saved to / loaded from a JSON-lines file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace cesim;

namespace {

std::mutex g_mu;
std::map<std::string, std::array<int, 3>> g_table;

std::string draw_key(cesim_ctx c) {
  char b[64];
  std::snprintf(b, sizeof(b), "drawAB p%d %dx%d", (int)c->prec, c->t1, c->t2);
  return b;
}

std::string gemm_key(cesim_ctx c, int R) {
  char b[96];
  std::snprintf(b, sizeof(b), "gemm s%d nu%d M%d n%d R%d", c->gemm_split, c->covd.nu_code,
                c->grid.m1 * c->grid.m2, (c->nobs + 511) / 512, (R + 255) / 256 * 256);
  return b;
}

bool lookup(const std::string& k, std::array<int, 3>& v) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_table.find(k);
  if (it == g_table.end()) return false;
  v = it->second;
  return true;
}

void store(const std::string& k, const std::array<int, 3>& v) {
  std::lock_guard<std::mutex> g(g_mu);
  g_table[k] = v;
}

// Accumulated ms of stage st over the timer's records since the last reset.
double stage_ms(StageTimer& t, int st) { return t.ms[st]; }

void reset_timer(StageTimer& t) {
  for (int i = 0; i < ST_COUNT; ++i) {
    t.ms[i] = 0;
    t.calls[i] = 0;
  }
}

}  // namespace

namespace cesim {

// A narrower pass-A column tile must beat the widest by this factor.
constexpr double kPassAMargin = 0.85;

DrawShape draw_shape(cesim_ctx c) {
  DrawShape d = c->draw_force;
  std::array<int, 3> v;
  if (lookup(draw_key(c), v)) {
    if (d.lcp < 0) d.lcp = v[0];
    if (d.rows == 0) d.rows = v[1];
  }
  return d;
}

int gemm_tile(cesim_ctx c, int R) {
  if (c->gemm_tile >= 1 && c->gemm_tile <= 5) return c->gemm_tile;
  std::array<int, 3> v;
  if (lookup(gemm_key(c, R), v) && v[0] >= 1 && v[0] <= 5) return v[0];
  return 1;
}

bool tune_has_entries(cesim_ctx c, int R) {
  std::array<int, 3> v;
  if (register_draw_path(c) && !lookup(draw_key(c), v)) return false;
  if (c->prec == CESIM_PREC_MIXED && c->nobs > 0 && !lookup(gemm_key(c, R), v)) return false;
  return true;
}

}  // namespace cesim

extern "C" {

cesim_status ce_autotune(cesim_ctx c, int nreal, void* fields) {
  if (!c || !fields || nreal < 1) return CESIM_ERR_INVALID_ARG;
  const int nt = std::min(nreal, 64);
  CESIM_HIP(hipStreamSynchronize(c->stream));
  c->timer.resolve();
  StageTimer saved_acc;
  std::copy(c->timer.ms, c->timer.ms + ST_COUNT, saved_acc.ms);
  std::copy(c->timer.calls, c->timer.calls + ST_COUNT, saved_acc.calls);
  const bool saved_on = c->timer.enabled;
  const DrawShape saved_force = c->draw_force;
  const int saved_tile = c->gemm_tile, saved_nreal = c->nreal;
  const bool saved_have = c->have_fields;
  cesim_status st = CESIM_OK;
  c->timer.enabled = true;
  auto timed = [&](auto&& launch, double out[3], const int stages[3]) -> cesim_status {
    CESIM_TRY(launch());                        // warm-up
    CESIM_HIP(hipStreamSynchronize(c->stream));
    c->timer.resolve();
    reset_timer(c->timer);
    for (int rep = 0; rep < 2; ++rep) CESIM_TRY(launch());
    CESIM_HIP(hipStreamSynchronize(c->stream));
    c->timer.resolve();
    for (int i = 0; i < 3; ++i) out[i] = stages[i] >= 0 ? stage_ms(c->timer, stages[i]) : 0.0;
    return CESIM_OK;
  };
  if (register_draw_path(c)) {
    c->draw_force = DrawShape{};
    const DrawShape mx = draw_shape_limits(c);
    const int st3[3] = {ST_DRAW_PASS_A, ST_DRAW_PASS_B, -1};
    double best[2] = {1e300, 1e300};
    std::array<int, 3> pick{mx.lcp, mx.rows, 0};
    std::vector<DrawShape> cands;
    for (int i = 0; i < 4; ++i) {
      const DrawShape d{std::max(0, mx.lcp - i), std::max(1, mx.rows >> i)};
      if (!cands.empty() && cands.back().lcp == d.lcp && cands.back().rows == d.rows) break;
      cands.push_back(d);
    }
    for (const DrawShape& d : cands) {
      c->draw_force = d;
      double ms[3];
      st = timed([&] { return ce_draw_device(c, nt, 0, 0, fields); }, ms, st3);
      if (st != CESIM_OK) break;
      const int v[2] = {d.lcp, d.rows};
      for (int q = 0; q < 2; ++q) {
        // Pass A with the widest column tile holds one workgroup per CU and
        // leaves LDS for the diagonal factorization kernel, which
        // condition() runs beside the draw; narrower tiles fill the LDS with
        // two workgroups and stall that chain.  Timed alone they can be a
        // few per cent faster, so they are taken only when clearly so.
        const double need = (q == 0 && best[q] < 1e300) ? kPassAMargin * best[q] : best[q];
        if (ms[q] < need) {
          best[q] = ms[q];
          pick[q] = v[q];
        }
      }
    }
    if (st == CESIM_OK) store(draw_key(c), pick);
  }
  if (st == CESIM_OK && c->prec == CESIM_PREC_MIXED && c->nobs > 0) {
    // the GEMM is timed at the full realization count (its key includes it);
    // its epilogue reads the prediction buffer, whose contents do not matter here
    st = krige_reserve(c, nreal);
    if (st == CESIM_OK)
      st = c->yhat.reserve(sizeof(float) * (size_t)c->grid.m1 * c->grid.m2);
    c->nreal = nreal;
    const int stg[3] = {ST_KRIGE_GEMM, -1, -1};
    double best = 1e300;
    int pick = 1;
    // candidates: the 256-realization tiles, the 512-realization tile above
    // 256 realizations, the 64- and 128-realization tiles up to 128
    std::vector<int> cands = {1, 2};
    if (nreal > 256) cands.push_back(3);
    if (nreal <= 128) cands.push_back(5);
    if (nreal <= 64) cands.push_back(4);
    for (int nf : cands) {
      if (st != CESIM_OK) break;
      c->gemm_tile = nf;
      double ms[3];
      st = timed([&] { return krige_grid_device(c, c->coef.as<double>(), fields); }, ms, stg);
      if (st == CESIM_OK && ms[0] < best) {
        best = ms[0];
        pick = nf;
      }
    }
    if (st == CESIM_OK) store(gemm_key(c, nreal), {pick, 0, 0});
  }
  (void)hipStreamSynchronize(c->stream);
  c->timer.resolve();
  std::copy(saved_acc.ms, saved_acc.ms + ST_COUNT, c->timer.ms);
  std::copy(saved_acc.calls, saved_acc.calls + ST_COUNT, c->timer.calls);
  c->timer.enabled = saved_on;
  c->draw_force = saved_force;
  c->gemm_tile = saved_tile;
  c->nreal = saved_nreal;
  c->have_fields = saved_have;
  return st;
}

int cesim_tune_entries(void) {
  std::lock_guard<std::mutex> g(g_mu);
  return (int)g_table.size();
}

void cesim_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_mu);
  g_table.clear();
}

cesim_status cesim_tune_save(const char* path) {
  if (!path) return CESIM_ERR_INVALID_ARG;
  std::FILE* f = std::fopen(path, "w");
  if (!f) return CESIM_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> g(g_mu);
    for (const auto& [k, v] : g_table)
      std::fprintf(f, "{\"key\": \"%s\", \"v\": [%d, %d, %d]}\n", k.c_str(), v[0], v[1], v[2]);
  }
  return std::fclose(f) == 0 ? CESIM_OK : CESIM_ERR_INVALID_ARG;
}

// Reads lines written by cesim_tune_save; entries replace existing ones.  A
// line that does not parse fails the call (entries before it are kept).
cesim_status cesim_tune_load(const char* path) {
  if (!path) return CESIM_ERR_INVALID_ARG;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return CESIM_ERR_INVALID_ARG;
  char line[512];
  cesim_status st = CESIM_OK;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '\n' || line[0] == 0) continue;
    char key[128];
    int a, b, c;
    if (std::sscanf(line, " {\"key\": \"%127[^\"]\", \"v\": [%d, %d, %d]}", key, &a, &b, &c) != 4 ||
        (std::strncmp(key, "drawAB ", 7) != 0 && std::strncmp(key, "gemm ", 5) != 0)) {
      st = CESIM_ERR_INVALID_ARG;
      break;
    }
    store(key, {a, b, c});
  }
  std::fclose(f);
  return st;
}

}  // extern "C"
