// C ABI of libscoup: argument validation, workspace layout, per-view launch
// sequence and the single status read-back per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <cmath>
#include <string>
#include <vector>

#include "scoup.h"
#include "scoup_internal.h"

using namespace scoup;

// Scratch of scoup_decode_noalloc: one array per GPU the library runs on,
// held until the process ends.  In host code the array's name is not a
// device address: the per-device address comes from hipGetSymbolAddress,
// taken once per device (with that device current) on the first call there.
constexpr size_t kDecodeScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kDecodeScratchBytes];

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

int tiles_of(int w, int h, int shift = 4) {
  const int t = 1 << shift;
  return ((w + t - 1) >> shift) * ((h + t - 1) >> shift);
}

// Workspace layout of one binning pass (+ the uplift's per-view offsets and records).
struct BinLayout {
  size_t status, vtot, splats, offsets, scan_part, tile_start, big_tiles, tile_order, bin_hist, radix_hist, tile_ids[2],
      keys[2], records, extra, total;
  unsigned int extra_cap;
  bool counting;
};

BinLayout bin_layout(int64_t n, int max_tiles, int64_t cap, int off_views, int rec_views, bool extra_entries) {
  BinLayout L{};
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  size_t off = 0;
  L.status = off; off = align256(off + sizeof(Status));
  L.vtot = off; off = align256(off + 8 * (size_t)kCountCams);
  L.splats = off; off = align256(off + sizeof(GSplat) * nn);
  L.offsets = off; off = align256(off + 4 * (size_t)(n + 1) * (size_t)off_views);
  const long long sparts =
      std::max(std::max(scan_blocks(n), scan_blocks(128 * radix_blocks(cap))), scan_blocks(max_tiles));
  L.scan_part = off; off = align256(off + 8 * (size_t)std::max<long long>(1, sparts));
  L.tile_start = off; off = align256(off + 4 * (size_t)(max_tiles + 1));
  L.big_tiles = off; off = align256(off + 4 * (size_t)max_tiles);
  L.tile_order = off; off = align256(off + 4 * (size_t)max_tiles);
  L.counting = count_binning_ok(n, max_tiles);
  L.bin_hist = off;
  if (L.counting) off = align256(off + 4 * (size_t)count_groups(n) * (size_t)max_tiles);
  L.radix_hist = off; off = align256(off + 4 * 128 * (size_t)std::max<long long>(1, radix_blocks(cap)));
  L.tile_ids[0] = off; off = align256(off + 4 * (size_t)cap);
  L.tile_ids[1] = off; off = align256(off + 4 * (size_t)cap);
  L.keys[0] = off; off = align256(off + 8 * (size_t)cap);
  L.keys[1] = off; off = align256(off + 8 * (size_t)cap);
  L.records = off; off = align256(off + 16 * (size_t)cap * (size_t)rec_views);
  // uplift: deferred weights of regions beyond a block's two record regions (one view at a time)
  L.extra_cap = extra_entries ? (unsigned int)std::max<int64_t>(1 << 18, std::min<int64_t>(cap / 16, 1 << 26)) : 0u;
  L.extra = off; off = align256(off + 16 * (size_t)L.extra_cap);
  L.total = off;
  return L;
}

// largest pair capacity whose single-view layout fits in `bytes` (0 if none)
int64_t capacity_for(int64_t n, int max_tiles, size_t bytes) {
  const size_t fixed = bin_layout(n, max_tiles, 0, 1, 0, false).total;
  if (bytes <= fixed + 8192) return 0;
  int64_t cap = (int64_t)(((bytes - fixed - 8192) * 8) / 197);
  while (cap > 0 && bin_layout(n, max_tiles, cap, 1, 0, false).total > bytes) cap -= 64;
  return std::min<int64_t>(std::max<int64_t>(cap, 0), 0x7fffffffLL);
}

// largest pair capacity whose single-view layout plus `per_pair` more bytes
// per pair fits in `bytes` (0 if none)
int64_t capacity_for_extra(int64_t n, int max_tiles, size_t bytes, size_t per_pair) {
  auto need = [&](int64_t cap) {
    return bin_layout(n, max_tiles, cap, 1, 0, false).total + align256(per_pair * (size_t)cap);
  };
  if (need(1) > bytes) return 0;
  int64_t lo = 1, hi = 0x7fffffffLL;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (need(mid) <= bytes) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// render backward: transposed codebook, dL/dW_hat map, dL/dC chunk partials
size_t render_bwd_fixed_bytes(size_t P, int m, int d) {
  return align256(decode_codebook_bytes(d, m, SCOUP_F32)) + align256(4 * P * (size_t)m) +
         align256(4 * (size_t)gemm_at_b_chunks((long long)P, m, d) * (size_t)m * (size_t)d);
}

int max_tiles_of(const scoup_views* v) {   // 8x8 blocks of the uplift
  int mt = 1;
  for (int i = 0; i < v->n_views; ++i) mt = std::max(mt, tiles_of(v->cams[i].width, v->cams[i].height, 3));
  return mt;
}

// The uplift keeps up to kLanes views in flight (binning of one overlapping
// the compositing of another) when a view batch holds two or more views:
// further sets of per-view binning buffers follow the first layout.
constexpr int kLanes = 4;                     // workspace sized for this many; the setting below may use fewer
int g_views_in_flight = kLanes;
struct TouchStats { uint64_t touches = 0, lost = 0, direct = 0, views = 0; };
TouchStats g_touch;                           // collected while stage timing is on
unsigned int g_extra_cap_limit = 0;           // 0: the layout's deferred-entry capacity
BinLayout uplift_layout(int64_t n, int mt, int64_t cap, int vb, int n_levels) {
  return bin_layout(n, mt, cap, vb, vb * n_levels, true);
}
BinLayout uplift_lane2_layout(int64_t n, int mt, int64_t cap) { return bin_layout(n, mt, cap, 0, 0, true); }
int uplift_lanes(int vb) { return std::max(1, std::min(g_views_in_flight, vb)); }
size_t uplift_layout_total(int64_t n, int mt, int64_t cap, int vb, int n_levels) {
  const size_t t = uplift_layout(n, mt, cap, vb, n_levels).total;
  const int lanes = std::max(1, std::min(kLanes, vb));
  return lanes > 1 ? align256(t) + (size_t)(lanes - 1) * align256(uplift_lane2_layout(n, mt, cap).total) : t;
}

// The library's further streams on the current device (default priority),
// and events ordering them against the caller's stream; created on first use.
struct SideStreams {
  hipStream_t s[kLanes - 1] = {};
  hipEvent_t start = nullptr, batch = nullptr;   // recorded on the caller's stream
  hipEvent_t done[kLanes - 1] = {};              // recorded on the library streams
};
std::mutex g_side_mu;
SideStreams g_side[64];
hipError_t side_streams(SideStreams** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_side_mu);
  SideStreams& ss = g_side[dev];
  if (!ss.start) {
    for (int k = 0; k < kLanes - 1; ++k) {
      if ((e = hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&ss.done[k], hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = hipEventCreateWithFlags(&ss.batch, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.start, hipEventDisableTiming)) != hipSuccess) return e;
  }
  *out = &ss;
  return hipSuccess;
}

void fill_bin(BinArgs& b, const scoup_gaussians* g, char* base, const BinLayout& L, long long capacity,
              int shift, int sort_cap) {
  b.means = g->means; b.log_scales = g->log_scales; b.quats = g->quats; b.opacities = g->opacities;
  b.n = g->n;
  b.tile_shift = shift;
  b.sort_cap = sort_cap;
  b.splats = reinterpret_cast<GSplat*>(base + L.splats);
  b.offsets = reinterpret_cast<unsigned int*>(base + L.offsets);
  b.scan_part = reinterpret_cast<unsigned long long*>(base + L.scan_part);
  b.tile_start = reinterpret_cast<unsigned int*>(base + L.tile_start);
  b.big_tiles = reinterpret_cast<unsigned int*>(base + L.big_tiles);
  b.tile_order = reinterpret_cast<unsigned int*>(base + L.tile_order);
  b.bin_hist = L.counting ? reinterpret_cast<unsigned int*>(base + L.bin_hist) : nullptr;
  b.radix_hist = reinterpret_cast<unsigned int*>(base + L.radix_hist);
  for (int k = 0; k < 2; ++k) {
    b.tile_ids[k] = reinterpret_cast<unsigned int*>(base + L.tile_ids[k]);
    b.keys[k] = reinterpret_cast<unsigned long long*>(base + L.keys[k]);
  }
  b.capacity = capacity;
  b.status = reinterpret_cast<Status*>(base + L.status);
  b.sorted = 0;
  b.pair_index = 0;
}

std::once_flag g_lds_once;
hipError_t g_lds_err = hipSuccess;
hipError_t ensure_lds_limits() {
  std::call_once(g_lds_once, [] {
    g_lds_err = render_set_lds_limits();
    if (g_lds_err == hipSuccess) g_lds_err = decode_set_lds_limits();
    if (g_lds_err == hipSuccess) g_lds_err = render_bwd_set_lds_limits();
    if (g_lds_err == hipSuccess) g_lds_err = binning_set_lds_limits();
  });
  return g_lds_err;
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
  if (!g_timer.on || stage < 0) return;
  hipEvent_t e = take_event();
  if (e) hipEventRecord(e, s);
  g_timer.open[stage] = e;
}
void StageTimer::end(int stage, hipStream_t s) {
  if (!g_timer.on || stage < 0) return;
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
  g_touch = TouchStats{};
  for (int i = 0; i < kNumStages; ++i) { g_timer.total_ms[i] = 0.0; g_timer.launches[i] = 0; }
}

int32_t scoup_stage_stats(int32_t stage, double* total_ms, int64_t* launches) {
  if (stage < 0 || stage >= kNumStages) return -1;
  if (total_ms) *total_ms = g_timer.total_ms[stage];
  if (launches) *launches = g_timer.launches[stage];
  return 0;
}


void scoup_uplift_touch_stats(uint64_t* touches, uint64_t* lost, uint64_t* direct, uint64_t* views) {
  if (touches) *touches = g_touch.touches;
  if (lost) *lost = g_touch.lost;
  if (direct) *direct = g_touch.direct;
  if (views) *views = g_touch.views;
}

void scoup_set_views_in_flight(int32_t k) { g_views_in_flight = std::max(1, std::min<int>(kLanes, k)); }

int32_t scoup_views_in_flight(void) { return g_views_in_flight; }

void scoup_set_deferred_entry_limit(int64_t n) {
  g_extra_cap_limit = n <= 0 ? 0u : (unsigned int)std::min<int64_t>(n, 0xffffffffLL);
}

const char* scoup_last_error(void) { return g_err.c_str(); }

const char* scoup_version(void) { return "libscoup 0.1 gfx950"; }

int64_t scoup_required_pair_capacity(void) { return g_required_pairs; }

size_t scoup_uplift_workspace_bytes(int64_t n_gaussians, const scoup_views* views, int64_t pair_capacity,
                                    int32_t view_batch) {
  return scoup_uplift_levels_workspace_bytes(n_gaussians, 1, views, pair_capacity, view_batch);
}

size_t scoup_uplift_levels_workspace_bytes(int64_t n_gaussians, int32_t n_levels, const scoup_views* levels,
                                           int64_t pair_capacity, int32_t view_batch) {
  if (!levels || n_gaussians < 0 || n_levels < 1 || n_levels > kMaxLevels) return 0;
  const scoup_views* views = &levels[0];
  if (views->n_views > 0 && !views->cams) return 0;
  if (pair_capacity <= 0) pair_capacity = std::max<int64_t>(6 * n_gaussians, 1 << 16);
  const int vb = std::max(1, std::min<int>(view_batch > 0 ? view_batch : views->n_views, views->n_views));
  return uplift_layout_total(n_gaussians, max_tiles_of(views), pair_capacity, vb, n_levels);
}

namespace {
scoup_status uplift_impl(const scoup_gaussians* g, int n_levels, const scoup_views* lvs, float* const* acc,
                         int32_t accumulate, int32_t k_top, int32_t* const* topk_idx, float* const* topk_val,
                         float* const* entropy, int64_t pair_capacity, int32_t view_batch, void* ws, size_t ws_bytes,
                         unsigned long long* n_contrib, void* stream) {
  scoup_status st = check_gaussians(g);
  if (st != SCOUP_OK) return st;
  if (!lvs) return fail(SCOUP_E_ARG, "views is NULL");
  if (n_levels < 1 || n_levels > kMaxLevels) return fail(SCOUP_E_ARG, "n_levels must be in [1, 4]");
  if (!acc) return fail(SCOUP_E_ARG, "acc array is NULL");
  const scoup_views* v = &lvs[0];
  for (int l = 0; l < n_levels; ++l) {
    if ((st = check_views(&lvs[l])) != SCOUP_OK) return st;
    const scoup_views& w = lvs[l];
    if (w.n_views != v->n_views || w.m_atoms != v->m_atoms)
      return fail(SCOUP_E_ARG, "all levels need the same views and m_atoms");
    for (int i = 0; i < w.n_views; ++i)
      if (w.cams[i].width != v->cams[i].width || w.cams[i].height != v->cams[i].height ||
          std::memcmp(&w.cams[i], &v->cams[i], sizeof(scoup_camera)) != 0)
        return fail(SCOUP_E_ARG, "all levels need the same cameras");
    if (w.n_views > 0 && w.region_base[w.n_views] > 0x7fffffffLL)
      return fail(SCOUP_E_ARG, "more than 2^31 regions in total");
    if (g->n > 0 && !acc[l]) return fail(SCOUP_E_ARG, "acc is NULL");
    if (k_top > 0 && g->n > 0 && (!topk_idx || !topk_val || !topk_idx[l] || !topk_val[l]))
      return fail(SCOUP_E_ARG, "Top-K arrays are NULL");
  }
  if (!ws) return fail(SCOUP_E_ARG, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace must be 256-byte aligned");
  if (pair_capacity < 1 || pair_capacity > 0x7fffffffLL) return fail(SCOUP_E_ARG, "pair_capacity out of range");
  const int vb = std::max(1, std::min<int>(view_batch > 0 ? view_batch : std::max(1, v->n_views),
                                           std::max(1, v->n_views)));
  const int mt = max_tiles_of(v);
  const BinLayout L = uplift_layout(g->n, mt, pair_capacity, vb, n_levels);
  const int lanes = uplift_lanes(vb);          // views in flight
  const size_t need = uplift_layout_total(g->n, mt, pair_capacity, vb, n_levels);
  if (ws_bytes < need) {
    g_required_pairs = pair_capacity;
    return fail(SCOUP_E_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes is smaller than the " +
                                       std::to_string(need) + " this capacity and view batch need");
  }
  HIP_TRY(ensure_lds_limits());
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  if (accumulate && g->n > 0 && v->n_views > 0) {
    // A resumed call must leave acc as it was if a view exceeds the pair
    // capacity: every view's pair count is found (one pass over the Gaussians
    // per kCountCams views, the projection's own box arithmetic) and checked
    // before anything is written.
    unsigned long long* vt = reinterpret_cast<unsigned long long*>(base + L.vtot);
    std::vector<unsigned long long> tot((size_t)v->n_views, 0ull);
    for (int v0 = 0; v0 < v->n_views; v0 += kCountCams) {
      CamBatch cb{};
      cb.n = std::min(kCountCams, v->n_views - v0);
      for (int j = 0; j < cb.n; ++j) cb.c[j] = to_dev(v->cams[v0 + j]);
      HIP_TRY(hipMemsetAsync(vt, 0, 8 * (size_t)kCountCams, s));
      HIP_TRY(launch_count_view_pairs(g->means, g->log_scales, g->quats, g->opacities, g->n, cb, 3, vt, s));
      HIP_TRY(hipMemcpyAsync(tot.data() + v0, vt, 8 * (size_t)cb.n, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    const unsigned long long mx = *std::max_element(tot.begin(), tot.end());
    if (mx > (unsigned long long)pair_capacity) {
      g_required_pairs = (int64_t)std::min<unsigned long long>(mx, 0x7fffffffull);
      return fail(SCOUP_E_WORKSPACE, "pair capacity " + std::to_string(pair_capacity) + " exceeded; need " +
                                         std::to_string(mx) + " (acc unchanged)");
    }
  }
  SideStreams* side = nullptr;
  if (lanes > 1) HIP_TRY(side_streams(&side));
  const BinLayout L2 = uplift_lane2_layout(g->n, mt, pair_capacity);
  char* lane_base[kLanes] = {base};
  for (int k = 1; k < lanes; ++k) lane_base[k] = base + align256(L.total) + (size_t)(k - 1) * align256(L2.total);
  Status* status[kLanes] = {};
  status[0] = reinterpret_cast<Status*>(base + L.status);
  for (int k = 1; k < lanes; ++k) status[k] = reinterpret_cast<Status*>(lane_base[k] + L2.status);
  for (int k = 0; k < lanes; ++k) HIP_TRY(hipMemsetAsync(status[k], 0, sizeof(Status), s));
  const size_t acc_bytes = sizeof(float) * (size_t)g->n * (size_t)v->m_atoms;
  if (!accumulate && acc_bytes)
    for (int l = 0; l < n_levels; ++l) HIP_TRY(hipMemsetAsync(acc[l], 0, acc_bytes, s));

  // lane k: binning buffers, status and deferred entries of the views it handles; views
  // go round the lanes, lane 0 on the caller's stream, the others on the library's streams
  UpliftViewArgs a[kLanes] = {};
  fill_bin(a[0].bin, g, base, L, pair_capacity, 3, kSortCap);
  a[0].extra = reinterpret_cast<float4*>(base + L.extra);
  a[0].extra_cap = g_extra_cap_limit ? std::min(L.extra_cap, g_extra_cap_limit) : L.extra_cap;
  for (int k = 1; k < lanes; ++k) {
    fill_bin(a[k].bin, g, lane_base[k], L2, pair_capacity, 3, kSortCap);
    a[k].extra = reinterpret_cast<float4*>(lane_base[k] + L2.extra);
    a[k].extra_cap = g_extra_cap_limit ? std::min(L2.extra_cap, g_extra_cap_limit) : L2.extra_cap;
  }
  unsigned int* off_all = a[0].bin.offsets;
  float2* rec_all = reinterpret_cast<float2*>(base + L.records);
  const size_t rec_view = 2 * (size_t)pair_capacity;           // float2 per view and level
  const bool stats = StageTimer::enabled();
  for (int k = 0; k < lanes; ++k) {
    a[k].count_touches = stats ? 1 : 0;
    a[k].n_levels = n_levels;
    a[k].m_atoms = v->m_atoms;
    for (int l = 0; l < n_levels; ++l) {
      a[k].lv[l].code_idx = lvs[l].code_idx; a[k].lv[l].code_val = lvs[l].code_val;
      a[k].lv[l].k_code = lvs[l].k_code; a[k].lv[l].acc = acc[l];
    }
  }
  hipStream_t strm[kLanes] = {s};
  for (int k = 1; k < lanes; ++k) strm[k] = side->s[k - 1];
  if (lanes > 1) {                            // the other lanes start after the clears above
    HIP_TRY(hipEventRecord(side->start, s));
    for (int k = 1; k < lanes; ++k) HIP_TRY(hipStreamWaitEvent(strm[k], side->start, 0));
  }
  const bool want_topk = k_top > 0;
  if (g->n > 0) {
    for (int v0 = 0; v0 < v->n_views; v0 += vb) {
      const int nvb = std::min(vb, v->n_views - v0);
      for (int j = 0; j < nvb; ++j) {
        const int i = v0 + j;
        UpliftViewArgs& av = a[j % lanes];
        BinArgs& b = av.bin;
        const scoup_camera& c = v->cams[i];
        b.cam = to_dev(c);
        b.tiles_x = (c.width + 7) / 8;
        b.n_tiles = tiles_of(c.width, c.height, 3);
        b.offsets = off_all + (size_t)j * (size_t)(g->n + 1);
        b.n_cull_records = n_levels;
        for (int l = 0; l < n_levels; ++l) {
          av.lv[l].records = rec_all + ((size_t)l * vb + j) * rec_view;
          b.cull_records[l] = av.lv[l].records;
          av.lv[l].rmap = lvs[l].region_maps + lvs[l].map_offsets[i];
          av.lv[l].n_regions = (int)(lvs[l].region_base[i + 1] - lvs[l].region_base[i]);
          av.lv[l].region_base = lvs[l].region_base[i];
        }
        HIP_TRY(launch_uplift_view(av, strm[j % lanes]));
      }
      for (int k = 1; k < lanes; ++k) {        // the row build reads the records of every lane
        HIP_TRY(hipEventRecord(side->done[k - 1], strm[k]));
        HIP_TRY(hipStreamWaitEvent(s, side->done[k - 1], 0));
      }
      const bool last = v0 + vb >= v->n_views;
      for (int l = 0; l < n_levels; ++l) {
        RowBuildArgs rb{};
        rb.n = g->n; rb.m_atoms = v->m_atoms; rb.k_code = lvs[l].k_code;
        rb.code_idx = lvs[l].code_idx; rb.code_val = lvs[l].code_val;
        rb.r_total = lvs[l].region_base[v->n_views];
        rb.offsets = off_all; rb.records = rec_all + (size_t)l * vb * rec_view; rb.capacity = pair_capacity;
        rb.acc = acc[l]; rb.status = status[0];
        rb.n_views = nvb;
        rb.k_top = (want_topk && last) ? k_top : 0;
        rb.topk_idx = want_topk ? topk_idx[l] : nullptr;
        rb.topk_val = want_topk ? topk_val[l] : nullptr;
        rb.entropy = (entropy && last) ? entropy[l] : nullptr;
        HIP_TRY(launch_rowbuild(rb, s));
      }
      if (lanes > 1 && !last) {                // the next batch reuses the records and offsets
        HIP_TRY(hipEventRecord(side->batch, s));
        for (int k = 1; k < lanes; ++k) HIP_TRY(hipStreamWaitEvent(strm[k], side->batch, 0));
      }
    }
    if (v->n_views == 0)
      for (int l = 0; l < n_levels; ++l) {
        if (want_topk) HIP_TRY(launch_topk(acc[l], g->n, v->m_atoms, k_top, topk_idx[l], topk_val[l], s));
        if (entropy && entropy[l]) HIP_TRY(launch_entropy(acc[l], g->n, v->m_atoms, entropy[l], s));
      }
  }
  Status hs[kLanes] = {};
  for (int k = 0; k < lanes; ++k) {
    if (n_contrib) HIP_TRY(launch_add_contrib(n_contrib, status[k], s));
    HIP_TRY(hipMemcpyAsync(&hs[k], status[k], sizeof(Status), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  Status h = hs[0];
  for (int k = 1; k < lanes; ++k) {
    h.any_overflow |= hs[k].any_overflow;
    h.max_pairs = std::max(h.max_pairs, hs[k].max_pairs);
    h.data_error |= hs[k].data_error;
  }
  if (stats && g->n > 0) {
    for (int k = 0; k < lanes; ++k) {
      g_touch.touches += hs[k].touches;
      g_touch.lost += hs[k].touch_lost;
      g_touch.direct += hs[k].n_direct;
    }
    g_touch.views += (uint64_t)v->n_views;
  }
  if (h.any_overflow) {
    g_required_pairs = (int64_t)h.max_pairs;
    return fail(SCOUP_E_WORKSPACE, "pair capacity " + std::to_string(pair_capacity) + " exceeded; need " +
                                       std::to_string(h.max_pairs));
  }
  if (h.data_error & 1u) return fail(SCOUP_E_DATA, "a region id is outside [-1, regions of its view)");
  if (h.data_error & 2u) return fail(SCOUP_E_DATA, "a code atom index is >= m_atoms");
  return SCOUP_OK;
}
}  // namespace

scoup_status scoup_uplift_accumulate(const scoup_gaussians* g, const scoup_views* v, float* acc,
                                     int32_t accumulate, int64_t pair_capacity, int32_t view_batch, void* ws,
                                     size_t ws_bytes, unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  float* accs[1] = {acc};
  return uplift_impl(g, 1, v, accs, accumulate, 0, nullptr, nullptr, nullptr, pair_capacity, view_batch, ws,
                     ws_bytes, n_contrib, stream);
}

scoup_status scoup_uplift_levels(const scoup_gaussians* g, int32_t n_levels, const scoup_views* levels, int32_t k,
                                 float* const* acc, int32_t* const* topk_idx, float* const* topk_val,
                                 float* const* entropy, int64_t pair_capacity, int32_t view_batch, void* ws, size_t ws_bytes,
                                 unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  if (!levels) return fail(SCOUP_E_ARG, "levels is NULL");
  if (k < 0 || k > 64 || k > levels[0].m_atoms) return fail(SCOUP_E_ARG, "k must be in [0, min(64, m_atoms)]");
  if (levels[0].m_atoms > 4096) return fail(SCOUP_E_ARG, "m_atoms must be <= 4096");
  return uplift_impl(g, n_levels, levels, acc, 0, k, topk_idx, topk_val, entropy, pair_capacity, view_batch, ws,
                     ws_bytes, n_contrib, stream);
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

size_t scoup_uplift_dense_workspace_bytes(int64_t n_gaussians, const scoup_views* views, int32_t dim,
                                          int64_t pair_capacity, int32_t view_batch) {
  if (!views || dim < 1) return 0;
  const int64_t rt = views->n_views > 0 ? views->region_base[views->n_views] : 0;
  return align256(4 * (size_t)rt * (size_t)dim) +
         scoup_uplift_levels_workspace_bytes(n_gaussians, 1, views, pair_capacity, view_batch);
}

scoup_status scoup_uplift_dense(const scoup_gaussians* g, const scoup_views* v, const float* codebook, int32_t dim,
                                float* features, float* z, int64_t pair_capacity, int32_t view_batch, void* ws,
                                size_t ws_bytes, unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  scoup_status st = check_gaussians(g);
  if (st != SCOUP_OK) return st;
  if ((st = check_views(v)) != SCOUP_OK) return st;
  if (dim < 1 || dim > 1024) return fail(SCOUP_E_ARG, "dim must be in [1, 1024]");
  if (!codebook || (g->n > 0 && (!features || !z))) return fail(SCOUP_E_ARG, "a dense uplift array is NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace NULL or misaligned");
  if (pair_capacity < 1 || pair_capacity > 0x7fffffffLL) return fail(SCOUP_E_ARG, "pair_capacity out of range");
  const long long rt = v->n_views > 0 ? v->region_base[v->n_views] : 0;
  const size_t fbytes = align256(4 * (size_t)rt * (size_t)dim);
  const int vb = std::max(1, std::min<int>(view_batch > 0 ? view_batch : std::max(1, v->n_views),
                                           std::max(1, v->n_views)));
  const BinLayout L = bin_layout(g->n, max_tiles_of(v), pair_capacity, vb, vb, true);
  if (ws_bytes < fbytes + L.total) {
    g_required_pairs = pair_capacity;
    return fail(SCOUP_E_WORKSPACE, "workspace too small for this capacity and view batch");
  }
  HIP_TRY(ensure_lds_limits());
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* fbase = static_cast<char*>(ws);
  float* F = reinterpret_cast<float*>(fbase);
  char* base = fbase + fbytes;
  Status* status = reinterpret_cast<Status*>(base + L.status);
  HIP_TRY(hipMemsetAsync(status, 0, sizeof(Status), s));
  if (g->n > 0) {
    HIP_TRY(hipMemsetAsync(features, 0, sizeof(float) * (size_t)g->n * dim, s));
    HIP_TRY(hipMemsetAsync(z, 0, sizeof(float) * (size_t)g->n, s));
  }
  HIP_TRY(launch_region_features(v->code_idx, v->code_val, rt, v->k_code, codebook, v->m_atoms, dim, F, status, s));
  UpliftViewArgs a{};
  BinArgs& b = a.bin;
  fill_bin(b, g, base, L, pair_capacity, 3, kSortCap);
  a.n_levels = 1;
  a.m_atoms = v->m_atoms;
  a.extra = reinterpret_cast<float4*>(base + L.extra);
  a.extra_cap = L.extra_cap;
  unsigned int* off_all = b.offsets;
  float2* rec_all = reinterpret_cast<float2*>(base + L.records);
  LevelView& lv = a.lv[0];
  lv.code_idx = v->code_idx; lv.code_val = v->code_val; lv.k_code = v->k_code;
  lv.acc = features; lv.dense_F = F; lv.dense_d = dim; lv.zsum = z;
  if (g->n > 0) {
    for (int v0 = 0; v0 < v->n_views; v0 += vb) {
      const int nvb = std::min(vb, v->n_views - v0);
      for (int j = 0; j < nvb; ++j) {
        const int i = v0 + j;
        const scoup_camera& c = v->cams[i];
        b.cam = to_dev(c);
        b.tiles_x = (c.width + 7) / 8;
        b.n_tiles = tiles_of(c.width, c.height, 3);
        b.offsets = off_all + (size_t)j * (size_t)(g->n + 1);
        lv.records = rec_all + (size_t)j * 2 * (size_t)pair_capacity;
        b.n_cull_records = 1;
        b.cull_records[0] = lv.records;
        lv.rmap = v->region_maps + v->map_offsets[i];
        lv.n_regions = (int)(v->region_base[i + 1] - v->region_base[i]);
        lv.region_base = v->region_base[i];
        HIP_TRY(launch_uplift_view(a, s));
      }
      const bool last = v0 + vb >= v->n_views;
      HIP_TRY(launch_rowbuild_dense(g->n, dim, F, rt, nvb, off_all, rec_all, pair_capacity, features, z, 1,
                                    last ? 1 : 0, s));
    }
    if (v->n_views == 0)
      HIP_TRY(launch_rowbuild_dense(g->n, dim, F, rt, 0, off_all, rec_all, pair_capacity, features, z, 1, 1, s));
  }
  if (n_contrib) HIP_TRY(launch_add_contrib(n_contrib, status, s));
  Status h{};
  HIP_TRY(hipMemcpyAsync(&h, status, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  if (h.any_overflow) {
    g_required_pairs = (int64_t)h.max_pairs;
    return fail(SCOUP_E_WORKSPACE, "pair capacity " + std::to_string(pair_capacity) + " exceeded; need " +
                                       std::to_string(h.max_pairs));
  }
  if (h.data_error & 1u) return fail(SCOUP_E_DATA, "a region id is outside [-1, regions of its view)");
  if (h.data_error & 2u) return fail(SCOUP_E_DATA, "a code atom index is >= m_atoms");
  return SCOUP_OK;
}

scoup_status scoup_entropy(const float* acc, int64_t n, int32_t m, float* out, void* stream) {
  g_err.clear();
  if (n < 0) return fail(SCOUP_E_ARG, "n < 0");
  if (m < 1) return fail(SCOUP_E_ARG, "m must be >= 1");
  if (n > 0 && (!acc || !out)) return fail(SCOUP_E_ARG, "an entropy array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_entropy(acc, n, m, out, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SCOUP_OK;
}

scoup_status scoup_uplift(const scoup_gaussians* g, const scoup_views* v, int32_t k, float* acc,
                          int32_t* topk_idx, float* topk_val, int64_t pair_capacity, int32_t view_batch, void* ws,
                          size_t ws_bytes, unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  if (!v) return fail(SCOUP_E_ARG, "views is NULL");
  if (k < 1 || k > 64 || k > v->m_atoms) return fail(SCOUP_E_ARG, "k must be in [1, min(64, m_atoms)]");
  if (v->m_atoms > 4096) return fail(SCOUP_E_ARG, "m_atoms must be <= 4096");
  if (g && g->n > 0 && (!topk_idx || !topk_val)) return fail(SCOUP_E_ARG, "Top-K arrays are NULL");
  float* accs[1] = {acc};
  int32_t* idxs[1] = {topk_idx};
  float* vals[1] = {topk_val};
  return uplift_impl(g, 1, v, accs, 0, k, idxs, vals, nullptr, pair_capacity, view_batch, ws, ws_bytes,
                     n_contrib, stream);
}

size_t scoup_render_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam, int64_t pair_capacity) {
  if (!cam || n_gaussians < 0) return 0;
  if (pair_capacity <= 0) pair_capacity = std::max<int64_t>(8 * n_gaussians, 1 << 16);
  return bin_layout(n_gaussians, tiles_of(cam->width, cam->height, 3), pair_capacity, 1, 0, false).total;
}

namespace {
// Render (and decode) of one camera; map / features / t_final optional; `prep`
// holds the converted codebook (NULL: no decode).
scoup_status render_impl(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val, int32_t k,
                         int32_t m_atoms, const scoup_camera* cam, void* coeff_map, scoup_dtype coeff_dtype,
                         float coeff_scale, float* t_final, const float* codebook, int32_t dim,
                         scoup_dtype in_dtype, void* features, scoup_dtype out_dtype, void* ws, size_t ws_bytes,
                         unsigned long long* n_contrib, void* stream) {
  scoup_status st = check_gaussians(g);
  if (st != SCOUP_OK) return st;
  if (!cam) return fail(SCOUP_E_ARG, "camera is NULL");
  if ((st = check_camera(*cam, "camera")) != SCOUP_OK) return st;
  if (k < 1 || k > 16) return fail(SCOUP_E_ARG, "k must be in [1, 16]");
  if (g->n * (int64_t)k >= (int64_t(1) << 30)) return fail(SCOUP_E_ARG, "n * k must be below 2^30");
  if (m_atoms < 1 || m_atoms > 512) return fail(SCOUP_E_ARG, "m_atoms must be in [1, 512]");
  if (g->n > 0 && (!topk_idx || !topk_val)) return fail(SCOUP_E_ARG, "Top-K arrays are NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace NULL or misaligned");
  const bool decode = codebook != nullptr;
  size_t pre = 0;
  if (decode) pre = 256 + align256(decode_codebook_bytes(m_atoms, dim, in_dtype));
  if (ws_bytes <= pre) return fail(SCOUP_E_WORKSPACE, "workspace smaller than the converted codebook");
  HIP_TRY(ensure_lds_limits());
  const int shift = 3;
  const int mt = tiles_of(cam->width, cam->height, shift);
  const long long capacity = capacity_for(g->n, mt, ws_bytes - pre);
  if (capacity < 1) {
    g_required_pairs = std::max<int64_t>(8 * g->n, 1 << 16);
    return fail(SCOUP_E_WORKSPACE, "workspace smaller than the fixed part");
  }
  const BinLayout L = bin_layout(g->n, mt, capacity, 1, 0, false);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  RenderBlockArgs a{};
  fill_bin(a.bin, g, base + pre, L, capacity, shift, kSortCap);
  a.bin.cam = to_dev(*cam);
  a.bin.tiles_x = (cam->width + 7) / 8;
  a.bin.n_tiles = mt;
  a.topk_idx = topk_idx; a.topk_val = topk_val; a.k = k; a.m_atoms = m_atoms;
  a.map = coeff_map; a.map_dtype = coeff_dtype; a.map_scale = coeff_scale; a.t_final = t_final;
  a.in_dtype = -1;
  a.out_dtype = out_dtype;
  if (decode) {
    float* scale = reinterpret_cast<float*>(base);
    void* prep = base + 256;
    HIP_TRY(launch_prep_codebook(codebook, m_atoms, dim, in_dtype, prep, scale, s, 0));
    a.in_dtype = in_dtype;
    a.codebook_prep = prep;
    a.cb_scale = in_dtype == SCOUP_FP8_E4M3 ? scale : nullptr;
    a.d = dim; a.kpad = decode_kpad(m_atoms, in_dtype); a.npad = decode_npad(dim);
    a.q_scale = in_dtype == SCOUP_FP8_E4M3 ? 256.0f : 1.0f;
    a.out_mul = 1.0f / a.q_scale;
    a.features = features;
  }
  Status* status = a.bin.status;
  HIP_TRY(hipMemsetAsync(status, 0, sizeof(Status), s));
  HIP_TRY(launch_render_block(a, s, kStRender));
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
  if (h.data_error & 4u) return fail(SCOUP_E_DATA, "a Top-K atom index is >= m_atoms");
  return SCOUP_OK;
}
}  // namespace

scoup_status scoup_render_coeff(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val,
                                int32_t k, int32_t m_atoms, const scoup_camera* cam, void* coeff_map,
                                scoup_dtype coeff_dtype, float coeff_scale, float* t_final, void* ws,
                                size_t ws_bytes, unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  if (coeff_dtype != SCOUP_F32 && coeff_dtype != SCOUP_BF16 && coeff_dtype != SCOUP_FP8_E4M3)
    return fail(SCOUP_E_ARG, "unknown coefficient dtype");
  if (!(coeff_scale > 0.f) || !std::isfinite(coeff_scale)) return fail(SCOUP_E_ARG, "coeff_scale must be > 0");
  if (!coeff_map) return fail(SCOUP_E_ARG, "coeff_map is NULL");
  return render_impl(g, topk_idx, topk_val, k, m_atoms, cam, coeff_map, coeff_dtype, coeff_scale, t_final, nullptr,
                     0, SCOUP_F32, nullptr, SCOUP_F32, ws, ws_bytes, n_contrib, stream);
}

size_t scoup_render_decode_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam, int32_t m_atoms,
                                           int32_t dim, scoup_dtype in_dtype, int64_t pair_capacity) {
  if (!cam || m_atoms < 1 || dim < 1) return 0;
  if (in_dtype != SCOUP_F32 && in_dtype != SCOUP_BF16 && in_dtype != SCOUP_FP8_E4M3) return 0;
  const size_t r = scoup_render_workspace_bytes(n_gaussians, cam, pair_capacity);
  return r ? 256 + align256(decode_codebook_bytes(m_atoms, dim, in_dtype)) + r : 0;
}

scoup_status scoup_render(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val, int32_t k,
                          const scoup_camera* cam, const float* codebook, int32_t m_atoms, int32_t dim,
                          scoup_dtype in_dtype, float* coeff_map, float* t_final, void* features,
                          scoup_dtype out_dtype, void* ws, size_t ws_bytes, unsigned long long* n_contrib,
                          void* stream) {
  g_err.clear();
  if (in_dtype != SCOUP_F32 && in_dtype != SCOUP_BF16 && in_dtype != SCOUP_FP8_E4M3)
    return fail(SCOUP_E_ARG, "unknown decode dtype");
  if (out_dtype != SCOUP_F32 && out_dtype != SCOUP_BF16) return fail(SCOUP_E_ARG, "output dtype must be F32 or BF16");
  if (dim < 1 || dim > 1024) return fail(SCOUP_E_UNSUPPORTED, "dim must be in [1, 1024]");
  if (!codebook || !features) return fail(SCOUP_E_ARG, "codebook or features is NULL");
  return render_impl(g, topk_idx, topk_val, k, m_atoms, cam, coeff_map, SCOUP_F32, 1.0f, t_final, codebook, dim,
                     in_dtype, features, out_dtype, ws, ws_bytes, n_contrib, stream);
}

size_t scoup_render_views_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam, int32_t n_views,
                                          int32_t m_atoms, int32_t dim, scoup_dtype in_dtype,
                                          int64_t pair_capacity) {
  if (n_views < 1) return 0;
  const size_t one = scoup_render_decode_workspace_bytes(n_gaussians, cam, m_atoms, dim, in_dtype, pair_capacity);
  if (!one) return 0;
  const size_t pre = 256 + align256(decode_codebook_bytes(m_atoms, dim, in_dtype));
  return pre + (size_t)std::min(kLanes, (int)n_views) * align256(one - pre);
}

// Several cameras of one size rendered as scoup_render does each, up to
// kLanes views in flight: view v runs on lane v mod lanes (the caller's
// stream or a library stream, each with its own set of binning buffers), so
// one view's projection and binning overlap another's render kernel.  The
// lanes share the converted codebook; one status read at the end.
scoup_status scoup_render_views(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val, int32_t k,
                                const scoup_camera* cams, int32_t n_views, const float* codebook, int32_t m_atoms,
                                int32_t dim, scoup_dtype in_dtype, void* features, scoup_dtype out_dtype, void* ws,
                                size_t ws_bytes, unsigned long long* n_contrib, void* stream) {
  g_err.clear();
  scoup_status st = check_gaussians(g);
  if (st != SCOUP_OK) return st;
  if (in_dtype != SCOUP_F32 && in_dtype != SCOUP_BF16 && in_dtype != SCOUP_FP8_E4M3)
    return fail(SCOUP_E_ARG, "unknown decode dtype");
  if (out_dtype != SCOUP_F32 && out_dtype != SCOUP_BF16) return fail(SCOUP_E_ARG, "output dtype must be F32 or BF16");
  if (dim < 1 || dim > 1024) return fail(SCOUP_E_UNSUPPORTED, "dim must be in [1, 1024]");
  if (n_views < 0) return fail(SCOUP_E_ARG, "n_views < 0");
  if (n_views == 0) return SCOUP_OK;
  if (!cams) return fail(SCOUP_E_ARG, "cameras is NULL");
  if (!codebook || !features) return fail(SCOUP_E_ARG, "codebook or features is NULL");
  for (int v = 0; v < n_views; ++v) {
    if ((st = check_camera(cams[v], "camera")) != SCOUP_OK) return st;
    if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
      return fail(SCOUP_E_ARG, "every camera must have the first camera's image size");
  }
  if (k < 1 || k > 16) return fail(SCOUP_E_ARG, "k must be in [1, 16]");
  if (g->n * (int64_t)k >= (int64_t(1) << 30)) return fail(SCOUP_E_ARG, "n * k must be below 2^30");
  if (m_atoms < 1 || m_atoms > 512) return fail(SCOUP_E_ARG, "m_atoms must be in [1, 512]");
  if (g->n > 0 && (!topk_idx || !topk_val)) return fail(SCOUP_E_ARG, "Top-K arrays are NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace NULL or misaligned");
  const size_t pre = 256 + align256(decode_codebook_bytes(m_atoms, dim, in_dtype));
  if (ws_bytes <= pre) return fail(SCOUP_E_WORKSPACE, "workspace smaller than the converted codebook");
  HIP_TRY(ensure_lds_limits());
  const int shift = 3;
  const int mt = tiles_of(cams[0].width, cams[0].height, shift);
  // the pair capacity depends on the view count only, not on the in-flight setting
  const int n_sets = std::min(kLanes, (int)n_views);
  const size_t set_bytes = ((ws_bytes - pre) / (size_t)n_sets) & ~(size_t)255;
  const long long capacity = capacity_for(g->n, mt, set_bytes);
  if (capacity < 1) {
    g_required_pairs = std::max<int64_t>(8 * g->n, 1 << 16);
    return fail(SCOUP_E_WORKSPACE, "workspace smaller than the fixed part");
  }
  const BinLayout L = bin_layout(g->n, mt, capacity, 1, 0, false);
  const int lanes = std::min(g_views_in_flight, n_sets);
  SideStreams* side = nullptr;
  if (lanes > 1) HIP_TRY(side_streams(&side));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipStream_t strm[kLanes] = {s};
  for (int j = 1; j < lanes; ++j) strm[j] = side->s[j - 1];
  char* base = static_cast<char*>(ws);
  float* scale = reinterpret_cast<float*>(base);
  void* prep = base + 256;
  HIP_TRY(launch_prep_codebook(codebook, m_atoms, dim, in_dtype, prep, scale, s, 0));
  RenderBlockArgs a[kLanes] = {};
  for (int j = 0; j < lanes; ++j) {
    RenderBlockArgs& aj = a[j];
    fill_bin(aj.bin, g, base + pre + (size_t)j * set_bytes, L, capacity, shift, kSortCap);
    aj.bin.tiles_x = (cams[0].width + 7) / 8;
    aj.bin.n_tiles = mt;
    aj.topk_idx = topk_idx; aj.topk_val = topk_val; aj.k = k; aj.m_atoms = m_atoms;
    aj.map = nullptr; aj.map_dtype = SCOUP_F32; aj.map_scale = 1.0f; aj.t_final = nullptr;
    aj.in_dtype = in_dtype;
    aj.codebook_prep = prep;
    aj.cb_scale = in_dtype == SCOUP_FP8_E4M3 ? scale : nullptr;
    aj.d = dim; aj.kpad = decode_kpad(m_atoms, in_dtype); aj.npad = decode_npad(dim);
    aj.q_scale = in_dtype == SCOUP_FP8_E4M3 ? 256.0f : 1.0f;
    aj.out_mul = 1.0f / aj.q_scale;
    aj.out_dtype = out_dtype;
    HIP_TRY(hipMemsetAsync(aj.bin.status, 0, sizeof(Status), s));
  }
  if (lanes > 1) {                            // the other lanes start after the codebook and the clears
    HIP_TRY(hipEventRecord(side->start, s));
    for (int j = 1; j < lanes; ++j) HIP_TRY(hipStreamWaitEvent(strm[j], side->start, 0));
  }
  const size_t view_bytes = (size_t)cams[0].width * (size_t)cams[0].height * (size_t)dim *
                            (out_dtype == SCOUP_F32 ? 4u : 2u);
  for (int v = 0; v < n_views; ++v) {
    RenderBlockArgs& av = a[v % lanes];
    av.bin.cam = to_dev(cams[v]);
    av.features = static_cast<char*>(features) + (size_t)v * view_bytes;
    HIP_TRY(launch_render_block(av, strm[v % lanes], kStRender));
  }
  for (int j = 1; j < lanes; ++j) {
    HIP_TRY(hipEventRecord(side->done[j - 1], strm[j]));
    HIP_TRY(hipStreamWaitEvent(s, side->done[j - 1], 0));
  }
  Status hs[kLanes] = {};
  for (int j = 0; j < lanes; ++j) {
    if (n_contrib) HIP_TRY(launch_add_contrib(n_contrib, a[j].bin.status, s));
    HIP_TRY(hipMemcpyAsync(&hs[j], a[j].bin.status, sizeof(Status), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  bool over = false;
  unsigned int need = 0, data = 0;
  for (int j = 0; j < lanes; ++j) {
    over = over || hs[j].any_overflow;
    need = std::max(need, hs[j].max_pairs);
    data |= hs[j].data_error;
  }
  if (over) {
    g_required_pairs = (int64_t)need;
    return fail(SCOUP_E_WORKSPACE, "pair capacity " + std::to_string(capacity) + " exceeded; need " +
                                       std::to_string(need));
  }
  if (data & 4u) return fail(SCOUP_E_DATA, "a Top-K atom index is >= m_atoms");
  return SCOUP_OK;
}

size_t scoup_decode_workspace_bytes(int32_t m_atoms, int32_t dim, scoup_dtype in_dtype) {
  if (m_atoms < 1 || dim < 1) return 0;
  return 256 + align256(decode_codebook_bytes(m_atoms, dim, in_dtype));
}

namespace {
// Eq. 8 with the converted codebook and its scale in `ws`; `stage` < 0 records no timing events.
scoup_status decode_impl(const void* coeff_map, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                         int32_t m_atoms, const float* codebook, int32_t dim, void* features, scoup_dtype out_dtype,
                         void* ws, size_t ws_bytes, void* stream, int stage) {
  if (in_dtype != SCOUP_F32 && in_dtype != SCOUP_BF16 && in_dtype != SCOUP_FP8_E4M3)
    return fail(SCOUP_E_ARG, "unknown input dtype");
  if (out_dtype != SCOUP_F32 && out_dtype != SCOUP_BF16) return fail(SCOUP_E_ARG, "output dtype must be F32 or BF16");
  if (n_pixels < 0) return fail(SCOUP_E_ARG, "n_pixels < 0");
  if (m_atoms < 1 || m_atoms > 4096) return fail(SCOUP_E_ARG, "m_atoms must be in [1, 4096]");
  if (dim < 1 || dim > 1024) return fail(SCOUP_E_UNSUPPORTED, "dim must be in [1, 1024]");
  if (!(coeff_scale > 0.f) || !std::isfinite(coeff_scale)) return fail(SCOUP_E_ARG, "coeff_scale must be > 0");
  if (!codebook || !features || (n_pixels > 0 && !coeff_map)) return fail(SCOUP_E_ARG, "a decode array is NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace NULL or misaligned");
  if (ws_bytes < scoup_decode_workspace_bytes(m_atoms, dim, in_dtype))
    return fail(SCOUP_E_WORKSPACE, "decode workspace too small");
  HIP_TRY(ensure_lds_limits());
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* scale = reinterpret_cast<float*>(base);
  void* prep = base + 256;
  HIP_TRY(launch_prep_codebook(codebook, m_atoms, dim, in_dtype, prep, scale, s, 0));
  DecodeArgs a{};
  a.coeff = coeff_map; a.P = n_pixels; a.m = m_atoms; a.d = dim; a.kpad = decode_kpad(m_atoms, in_dtype);
  a.in_dtype = in_dtype; a.out_dtype = out_dtype; a.codebook_prep = prep;
  a.cb_scale = in_dtype == SCOUP_FP8_E4M3 ? scale : nullptr;
  a.out_mul = 1.0f / coeff_scale;
  a.out = features;
  HIP_TRY(launch_decode(a, s, stage));
  HIP_TRY(hipStreamSynchronize(s));
  if (stage >= 0) StageTimer::collect();
  return SCOUP_OK;
}

// the address of this GPU's copy of `scratch` (below the namespace)
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

hipError_t decode_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

scoup_status scoup_decode(const void* coeff_map, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                          int32_t m_atoms, const float* codebook, int32_t dim, void* features,
                          scoup_dtype out_dtype, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  return decode_impl(coeff_map, in_dtype, coeff_scale, n_pixels, m_atoms, codebook, dim, features, out_dtype, ws,
                     ws_bytes, stream, kStDecode);
}

size_t scoup_decode_noalloc_max_bytes(void) { return kDecodeScratchBytes; }

scoup_status scoup_decode_noalloc(const void* coeff_map, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                                  int32_t m_atoms, const float* codebook, int32_t dim, void* features,
                                  scoup_dtype out_dtype, void* stream) {
  g_err.clear();
  if (m_atoms >= 1 && dim >= 1 &&
      scoup_decode_workspace_bytes(m_atoms, dim, in_dtype) > kDecodeScratchBytes)
    return fail(SCOUP_E_ARG, "codebook of " + std::to_string(m_atoms) + " x " + std::to_string(dim) +
                                 " needs more than the " + std::to_string(kDecodeScratchBytes) +
                                 " bytes of scratch of scoup_decode_noalloc; use scoup_decode");
  void* ws = nullptr;
  HIP_TRY(decode_scratch(&ws));
  return decode_impl(coeff_map, in_dtype, coeff_scale, n_pixels, m_atoms, codebook, dim, features, out_dtype, ws,
                     kDecodeScratchBytes, stream, -1);
}

size_t scoup_relevancy_workspace_bytes(int32_t m_atoms, int32_t n_queries, scoup_dtype in_dtype) {
  if (m_atoms < 1 || m_atoms > 4096 || n_queries < 1 || n_queries > 1024) return 0;
  if (in_dtype != SCOUP_F32 && in_dtype != SCOUP_BF16 && in_dtype != SCOUP_FP8_E4M3) return 0;
  return align256(relevancy_frag_bytes(m_atoms, n_queries, in_dtype));
}

scoup_status scoup_relevancy(const void* coeff, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                             int32_t m_atoms, const float* codebook, int32_t dim, const float* queries,
                             int32_t n_queries, const float* canon, int32_t n_canon, float temperature,
                             float* scores, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (in_dtype != SCOUP_F32 && in_dtype != SCOUP_BF16 && in_dtype != SCOUP_FP8_E4M3)
    return fail(SCOUP_E_ARG, "unknown input dtype");
  if (n_pixels < 0) return fail(SCOUP_E_ARG, "n_pixels < 0");
  if (m_atoms < 1 || m_atoms > 4096) return fail(SCOUP_E_ARG, "m_atoms must be in [1, 4096]");
  if (dim < 1 || dim > 4096) return fail(SCOUP_E_ARG, "dim must be in [1, 4096]");
  if (n_queries < 1 || n_queries > 1024) return fail(SCOUP_E_ARG, "n_queries must be in [1, 1024]");
  if (n_canon < 1 || n_canon > 4) return fail(SCOUP_E_ARG, "n_canon must be in [1, 4]");
  if (!(temperature > 0.f) || !std::isfinite(temperature)) return fail(SCOUP_E_ARG, "temperature must be > 0");
  if (!(coeff_scale > 0.f) || !std::isfinite(coeff_scale)) return fail(SCOUP_E_ARG, "coeff_scale must be > 0");
  if (!codebook || !queries || !canon || (n_pixels > 0 && (!coeff || !scores)))
    return fail(SCOUP_E_ARG, "a relevancy array is NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace NULL or misaligned");
  if (ws_bytes < scoup_relevancy_workspace_bytes(m_atoms, n_queries, in_dtype))
    return fail(SCOUP_E_WORKSPACE, "relevancy workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RelevancyArgs a{};
  a.coeff = coeff; a.P = n_pixels; a.m = m_atoms; a.d = dim; a.in_dtype = in_dtype;
  a.codebook = codebook; a.queries = queries; a.canon = canon; a.Q = n_queries; a.n_canon = n_canon;
  a.temperature = temperature; a.out_mul = 1.0f / coeff_scale; a.frag = ws; a.out = scores;
  HIP_TRY(launch_relevancy(a, s));
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  return SCOUP_OK;
}

size_t scoup_render_backward_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam, int32_t m_atoms,
                                              int32_t dim, int64_t pair_capacity) {
  if (!cam || n_gaussians < 0 || m_atoms < 1 || dim < 1 || cam->width <= 0 || cam->height <= 0) return 0;
  const size_t P = (size_t)cam->width * cam->height;
  if (pair_capacity <= 0) pair_capacity = std::max<int64_t>(16 * n_gaussians, 1 << 16);
  const int mt = tiles_of(cam->width, cam->height, 3);
  return render_bwd_fixed_bytes(P, m_atoms, dim) + bin_layout(n_gaussians, mt, pair_capacity, 1, 0, false).total +
         align256(4 * (size_t)kBwdKMax * (size_t)pair_capacity);
}

scoup_status scoup_render_backward(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val,
                                   int32_t k, int32_t m_atoms, const scoup_camera* cam, const float* coeff_map,
                                   const float* codebook, int32_t dim, const float* grad_features,
                                   float* grad_topk_val, float* grad_codebook, void* ws, size_t ws_bytes,
                                   void* stream) {
  g_err.clear();
  scoup_status st = check_gaussians(g);
  if (st != SCOUP_OK) return st;
  if (!cam) return fail(SCOUP_E_ARG, "camera is NULL");
  if ((st = check_camera(*cam, "camera")) != SCOUP_OK) return st;
  if (k < 1 || k > kBwdKMax) return fail(SCOUP_E_ARG, "k must be in [1, 16]");
  if (m_atoms < 1 || m_atoms > 512) return fail(SCOUP_E_ARG, "m_atoms must be in [1, 512]");
  if (dim < 1 || dim > 4096) return fail(SCOUP_E_ARG, "dim must be in [1, 4096]");
  if (!coeff_map || !codebook || !grad_features || !grad_codebook)
    return fail(SCOUP_E_ARG, "a backward array is NULL");
  if (g->n > 0 && (!topk_idx || !topk_val || !grad_topk_val)) return fail(SCOUP_E_ARG, "Top-K arrays are NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SCOUP_E_ARG, "workspace NULL or misaligned");
  HIP_TRY(ensure_lds_limits());
  const long long P = (long long)cam->width * cam->height;
  const size_t prep_b = align256(decode_codebook_bytes(dim, m_atoms, SCOUP_F32));
  const size_t dw_b = align256(4 * (size_t)P * m_atoms);
  const size_t fixed = render_bwd_fixed_bytes((size_t)P, m_atoms, dim);
  const int shift = 3;
  const int mt = tiles_of(cam->width, cam->height, shift);
  const long long capacity =
      ws_bytes > fixed ? capacity_for_extra(g->n, mt, ws_bytes - fixed, 4 * (size_t)kBwdKMax) : 0;
  if (capacity < 1) {
    g_required_pairs = std::max<int64_t>(16 * g->n, 1 << 16);
    return fail(SCOUP_E_WORKSPACE, "workspace smaller than the fixed part");
  }
  const BinLayout L = bin_layout(g->n, mt, capacity, 1, 0, false);
  char* base = static_cast<char*>(ws);
  void* prep = base;
  float* dW = reinterpret_cast<float*>(base + prep_b);
  float* gemm_part = reinterpret_cast<float*>(base + prep_b + dw_b);
  char* bbase = base + fixed;
  float* pair_part = reinterpret_cast<float*>(bbase + L.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RenderBwdArgs a{};
  fill_bin(a.bin, g, bbase, L, capacity, shift, kSortCap);
  a.bin.cam = to_dev(*cam);
  a.bin.tiles_x = (cam->width + 7) / 8;
  a.bin.n_tiles = mt;
  a.bin.pair_index = 1;
  a.topk_idx = topk_idx; a.topk_val = topk_val; a.k = k; a.m_atoms = m_atoms;
  a.dW = dW; a.pair_part = pair_part; a.grad_val = grad_topk_val;
  Status* status = a.bin.status;
  HIP_TRY(hipMemsetAsync(status, 0, sizeof(Status), s));
  // binning first: its pair-capacity check gates every write to the caller's gradients
  HIP_TRY(launch_bin_view(a.bin, s));
  // dW = G C^T : K = dim, N = m_atoms, B(k, n) = C[n * dim + k]
  HIP_TRY(launch_prep_codebook(codebook, dim, m_atoms, SCOUP_F32, prep, nullptr, s, 1));
  DecodeArgs d{};
  d.coeff = grad_features; d.P = P; d.m = dim; d.d = m_atoms; d.kpad = decode_kpad(dim, SCOUP_F32);
  d.in_dtype = SCOUP_F32; d.out_dtype = SCOUP_F32; d.codebook_prep = prep; d.cb_scale = nullptr;
  d.out_mul = 1.0f; d.out = dW; d.ldo = m_atoms;
  HIP_TRY(launch_decode(d, s, kStBwdGemm));
  HIP_TRY(launch_gemm_at_b(coeff_map, grad_features, P, m_atoms, dim, gemm_part, grad_codebook, status, s));
  HIP_TRY(launch_render_bwd_view(a, s));
  Status h{};
  HIP_TRY(hipMemcpyAsync(&h, status, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  StageTimer::collect();
  if (h.any_overflow) {
    g_required_pairs = (int64_t)h.max_pairs;
    return fail(SCOUP_E_WORKSPACE, "pair capacity " + std::to_string(capacity) + " exceeded; need " +
                                       std::to_string(h.max_pairs) + " (gradients unchanged)");
  }
  return SCOUP_OK;
}

}  // extern "C"
