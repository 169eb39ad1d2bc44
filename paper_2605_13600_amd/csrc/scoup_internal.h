// Host-side launcher interface between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "scoup_device.h"

namespace scoup {

enum Stage { kStProject = 0, kStScan, kStEmit, kStSortBig, kStComposite, kStTopk, kStRender, kStDecode,
             kStRenderBwd, kStBwdGemm, kNumStages };

// Records a HIP event pair around each launch when stage timing is enabled.
struct StageTimer {
  static bool enabled();
  static void begin(int stage, hipStream_t s);
  static void end(int stage, hipStream_t s);
  static void collect();   // after the stream is synchronised
};

struct UpliftViewArgs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacities;
  long long n;
  CamDev cam;
  int tiles_x, n_tiles;
  GSplat* splats;
  unsigned int* tile_count;
  unsigned int* tile_cursor;
  unsigned int* tile_start;
  unsigned long long* keys;
  long long capacity;
  const int* rmap;
  int n_regions;
  long long region_base;
  const int* code_idx;
  const float* code_val;
  int k_code, m_atoms;
  float* acc;
  Status* status;
};

hipError_t launch_uplift_view(const UpliftViewArgs& a, hipStream_t s);
hipError_t launch_topk(const float* acc, long long n, int m, int k, int* idx, float* val, hipStream_t s);
hipError_t launch_add_contrib(unsigned long long* dst, const Status* st, hipStream_t s);

}  // namespace scoup
