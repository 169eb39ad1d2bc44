// C ABI of libscoup: argument validation, workspace layout, per-view launch
// sequence and the single status read-back per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "scoup.h"
#include "scoup_internal.h"

using namespace scoup;

namespace {

thread_local std::string g_err;
thread_local int64_t g_required_pairs = 0;

scoup_status fail(scoup_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(x)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(SCOUP_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct UpliftLayout {
  size_t splats, tile_count, tile_cursor, tile_start, status, keys;
  size_t fixed;        // bytes before the key array
  int max_tiles;
};

int tiles_of(int w, int h) { return ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile); }

UpliftLayout uplift_layout(int64_t n, const scoup_views* v) {
  UpliftLayout L{};
  int mt = 1;
  for (int i = 0; i < v->n_views; ++i) mt = std::max(mt, tiles_of(v->cams[i].width, v->cams[i].height));
  L.max_tiles = mt;
  size_t off = 0;
  L.status = off; off = align256(off + sizeof(Status));
  L.splats = off; off = align256(off + sizeof(GSplat) * (size_t)std::max<int64_t>(n, 1));
  L.tile_count = off; off = align256(off + 4 * (size_t)mt);
  L.tile_cursor = off; off = align256(off + 4 * (size_t)mt);
  L.tile_start = off; off = align256(off + 4 * (size_t)(mt + 1));
  L.keys = off;
  L.fixed = off;
  return L;
}

scoup_status check_gaussians(const scoup_gaussians* g) {
  if (!g) return fail(SCOUP_E_ARG, "gaussians is NULL");
  if (g->n < 0 || g->n > 0x7fffffffLL) return fail(SCOUP_E_ARG, "gaussian count out of range [0, 2^31)");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacities))
    return fail(SCOUP_E_ARG, "a gaussian array is NULL");
  return SCOUP_OK;
}

scoup_status check_camera(const scoup_camera& c, const char* what) {
  if (c.width <= 0 || c.height <= 0 || c.width > 32767 || c.height > 32767)
    return fail(SCOUP_E_ARG, std::string(what) + ": image size must be in [1, 32767]");
  if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(SCOUP_E_ARG, std::string(what) + ": fx, fy must be > 0");
  if (!(c.near_z > 0.f)) return fail(SCOUP_E_ARG, std::string(what) + ": near_z must be > 0");
  return SCOUP_OK;
}

scoup_status check_views(const scoup_views* v) {
  if (!v) return fail(SCOUP_E_ARG, "views is NULL");
  if (v->n_views < 0) return fail(SCOUP_E_ARG, "n_views < 0");
  if (v->m_atoms < 1) return fail(SCOUP_E_ARG, "m_atoms must be >= 1");
  if (v->k_code < 1) return fail(SCOUP_E_ARG, "k_code must be >= 1");
  if (v->n_views == 0) return SCOUP_OK;
  if (!v->cams || !v->region_maps || !v->map_offsets || !v->region_base)
    return fail(SCOUP_E_ARG, "a view array is NULL");
  for (int i = 0; i < v->n_views; ++i) {
    scoup_status s = check_camera(v->cams[i], "camera");
    if (s != SCOUP_OK) return s;
    const int64_t hw = (int64_t)v->cams[i].width * v->cams[i].height;
    if (v->map_offsets[i + 1] - v->map_offsets[i] != hw)
      return fail(SCOUP_E_ARG, "map_offsets do not match the camera image sizes");
    if (v->region_base[i + 1] < v->region_base[i]) return fail(SCOUP_E_ARG, "region_base must be non-decreasing");
    if (v->region_base[i + 1] - v->region_base[i] > 0x7fffffffLL) return fail(SCOUP_E_ARG, "too many regions");
  }
  if (v->region_base[0] < 0) return fail(SCOUP_E_ARG, "region_base[0] < 0");
  if (v->region_base[v->n_views] > v->region_base[0] && (!v->code_idx || !v->code_val))
    return fail(SCOUP_E_ARG, "code arrays are NULL");
  return SCOUP_OK;
}

CamDev to_dev(const scoup_camera& c) {
  CamDev d;
  std::memcpy(d.R, c.R, sizeof d.R);
  std::memcpy(d.t, c.t, sizeof d.t);
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  d.width = c.width; d.height = c.height; d.near_z = c.near_z;
  return d;
}

struct TimerState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  hipEvent_t open[kNumStages] = {};
  double total_ms[kNumStages] = {};
  long long launches[kNumStages] = {};
};
TimerState g_timer;

hipEvent_t take_event() {
  if (!g_timer.pool.empty()) {
    hipEvent_t e = g_timer.pool.back();
    g_timer.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

namespace scoup {
bool StageTimer::enabled() { return g_timer.on; }
void StageTimer::begin(int stage, hipStream_t s) {
  if (!g_timer.on) return;
  hipEvent_t e = take_event();
  if (e) hipEventRecord(e, s);
  g_timer.open[stage] = e;
}
void StageTimer::end(int stage, hipStream_t s) {
  if (!g_timer.on) return;
  hipEvent_t b = g_timer.open[stage];
  g_timer.open[stage] = nullptr;
  hipEvent_t e = take_event();
  if (!b || !e) return;
  hipEventRecord(e, s);
  g_timer.pending.push_back({stage, {b, e}});
}
void StageTimer::collect() {
  for (auto& p : g_timer.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
      g_timer.total_ms[p.first] += ms;
      g_timer.launches[p.first] += 1;
    }
    g_timer.pool.push_back(p.second.first);
    g_timer.pool.push_back(p.second.second);
  }
  g_timer.pending.clear();
}
}  // namespace scoup

extern "C" {

void scoup_stage_timing(int32_t enable) {
  g_timer.on = enable != 0;
  for (int i = 0; i < kNumStages; ++i) { g_timer.total_ms[i] = 0.0; g_timer.launches[i] = 0; }
}

int32_t scoup_stage_stats(int32_t stage, double* total_ms, int64_t* launches) {
  if (stage < 0 || stage >= kNumStages) return -1;
  if (total_ms) *total_ms = g_timer.total_ms[stage];
  if (launches) *launches = g_timer.launches[stage];
  return 0;
}


const char* scoup_last_error(void) { return g_err.c_str(); }

const char* scoup_version(void) { return "libscoup 0.1 gfx950"; }

int64_t scoup_required_pair_capacity(void) { return g_required_pairs; }

size_t scoup_uplift_workspace_bytes(int64_t n_gaussians, const scoup_views* views, int64_t pair_capacity) {
  if (!views || n_gaussians < 0) return 0;
  if (views->n_views > 0 && !views->cams) return 0;
  UpliftLayout L = uplift_layout(n_gaussians, views);
  if (pair_capacity <= 0) pair_capacity = std::max<int64_t>(8 * n_gaussians, 1 << 16);
  return L.fixed + align256(8 * (size_t)pair_capacity);
}

scoup_status scoup_uplift_accumulate(const scoup_gaussians* g, const scoup_views* v, float* acc,
                                     int32_t accumulate, void* ws, size_t ws_bytes,
                                     unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  scoup_status st = check_gaussians(g);
  if (st != SCOUP_OK) return st;
  if ((st = check_views(v)) != SCOUP_OK) return st;
  if (g->n > 0 && !acc) return fail(SCOUP_E_ARG, "acc is NULL");
  if (!ws) return fail(SCOUP_E_ARG, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace must be 256-byte aligned");
  const UpliftLayout L = uplift_layout(g->n, v);
  if (ws_bytes < L.fixed + 8 * 1024) {
    g_required_pairs = std::max<int64_t>(8 * g->n, 1 << 16);
    return fail(SCOUP_E_WORKSPACE, "workspace smaller than the fixed part");
  }
  long long capacity = (long long)((ws_bytes - L.fixed) / 8);
  capacity = std::min<long long>(capacity, 0x7fffffffLL);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  Status* status = reinterpret_cast<Status*>(base + L.status);
  HIP_TRY(hipMemsetAsync(status, 0, sizeof(Status), s));
  HIP_TRY(hipMemsetAsync(base + L.tile_count, 0, 4 * (size_t)L.max_tiles, s));
  const size_t acc_bytes = sizeof(float) * (size_t)g->n * (size_t)v->m_atoms;
  if (!accumulate && acc_bytes) HIP_TRY(hipMemsetAsync(acc, 0, acc_bytes, s));

  UpliftViewArgs a{};
  a.means = g->means; a.log_scales = g->log_scales; a.quats = g->quats; a.opacities = g->opacities;
  a.n = g->n;
  a.splats = reinterpret_cast<GSplat*>(base + L.splats);
  a.tile_count = reinterpret_cast<unsigned int*>(base + L.tile_count);
  a.tile_cursor = reinterpret_cast<unsigned int*>(base + L.tile_cursor);
  a.tile_start = reinterpret_cast<unsigned int*>(base + L.tile_start);
  a.keys = reinterpret_cast<unsigned long long*>(base + L.keys);
  a.capacity = capacity;
  a.code_idx = v->code_idx; a.code_val = v->code_val;
  a.k_code = v->k_code; a.m_atoms = v->m_atoms;
  a.acc = acc;
  a.status = status;
  for (int i = 0; i < v->n_views; ++i) {
    const scoup_camera& c = v->cams[i];
    a.cam = to_dev(c);
    a.tiles_x = (c.width + kTile - 1) / kTile;
    a.n_tiles = tiles_of(c.width, c.height);
    a.rmap = v->region_maps + v->map_offsets[i];
    a.n_regions = (int)(v->region_base[i + 1] - v->region_base[i]);
    a.region_base = v->region_base[i];
    HIP_TRY(launch_uplift_view(a, s));
  }
  if (n_contrib) HIP_TRY(launch_add_contrib(n_contrib, status, s));
  Status h{};
  HIP_TRY(hipMemcpyAsync(&h, status, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  if (h.any_overflow) {
    g_required_pairs = (int64_t)h.max_pairs;
    return fail(SCOUP_E_WORKSPACE, "pair capacity " + std::to_string(capacity) + " exceeded; need " +
                                       std::to_string(h.max_pairs));
  }
  if (h.data_error & 1u) return fail(SCOUP_E_DATA, "a region id is outside [-1, regions of its view)");
  if (h.data_error & 2u) return fail(SCOUP_E_DATA, "a code atom index is >= m_atoms");
  return SCOUP_OK;
}

scoup_status scoup_topk(const float* acc, int64_t n, int32_t m, int32_t k, int32_t* idx, float* val,
                        void* stream) {
  g_err.clear();
  if (n < 0) return fail(SCOUP_E_ARG, "n < 0");
  if (m < 1 || m > 4096) return fail(SCOUP_E_ARG, "m must be in [1, 4096]");
  if (k < 1 || k > 64 || k > m) return fail(SCOUP_E_ARG, "k must be in [1, min(64, m)]");
  if (n > 0 && (!acc || !idx || !val)) return fail(SCOUP_E_ARG, "a Top-K array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_topk(acc, n, m, k, idx, val, s));
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  return SCOUP_OK;
}

scoup_status scoup_uplift(const scoup_gaussians* g, const scoup_views* v, int32_t k, float* acc,
                          int32_t* topk_idx, float* topk_val, void* ws, size_t ws_bytes,
                          unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  if (!v) return fail(SCOUP_E_ARG, "views is NULL");
  if (k < 1 || k > 64 || k > v->m_atoms) return fail(SCOUP_E_ARG, "k must be in [1, min(64, m_atoms)]");
  if (v->m_atoms > 4096) return fail(SCOUP_E_ARG, "m_atoms must be <= 4096");
  scoup_status st = scoup_uplift_accumulate(g, v, acc, 0, ws, ws_bytes, n_contrib, stream);
  if (st != SCOUP_OK) return st;
  return scoup_topk(acc, g->n, v->m_atoms, k, topk_idx, topk_val, stream);
}

}  // extern "C"
