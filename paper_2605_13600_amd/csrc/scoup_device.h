// Device-side types and helpers shared by the libscoup kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scoup.h"

namespace scoup {

constexpr int kTile = 16;            // screen tile edge (pixels); 4 waves of 8x8 per tile
constexpr int kTileThreads = 256;
constexpr int kSortCap = 4096;       // tile lists up to this length are sorted in LDS
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// Per (view, Gaussian) projected splat, 48 bytes, 16-byte aligned.
// mu2d = (ix + fx, iy + fy) with ix = floor(mu2d.x), fx in [0,1): keeping the
// integer part exact holds pixel offsets to ~1e-7 px at any image size.
// The conic (inverse dilated 2D covariance) is stored as the scaled factor L
// with d^T conic d * log2(e)/2 = (l00 dx + l10 dy)^2 + (l11 dy)^2, so
// alpha = o * exp2(-q) with q a sum of squares (never negative, no cancellation).
// bbox: inclusive pixel box (x0, x1, y0, y1) clamped to the image containing
// every pixel where alpha can reach 1/255 (widened by one pixel).
struct __align__(16) GSplat {
  int ix, iy;
  float fx, fy;
  float l00, l10, l11, opacity;
  int16_t bx0, bx1, by0, by1;
  uint32_t depth_bits;   // float32 view depth (positive, so bits order like values)
  uint32_t pad;
};
static_assert(sizeof(GSplat) == 48, "GSplat layout");

// Small per-call status block in the workspace.
struct Status {
  unsigned int total_pairs;     // pairs of the current view
  unsigned int view_overflow;   // current view exceeded the pair capacity
  unsigned int any_overflow;
  unsigned int max_pairs;       // largest per-view pair count seen
  unsigned int data_error;      // region id out of range
  unsigned int pad[3];
  unsigned long long contrib;   // contributions composited
};

struct CamDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int width, height;
  float near_z;
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace scoup
