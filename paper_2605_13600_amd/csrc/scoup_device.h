// Device-side types and helpers shared by the libscoup kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scoup.h"

namespace scoup {

constexpr int kTile = 16;            // screen tile edge (pixels); 4 waves of 8x8 per tile
constexpr int kTileThreads = 256;
constexpr int kSortCap = 4096;       // block lists up to this length are sorted in LDS (k_sort_blocks)
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
  uint32_t depth_bits;   // float32 view depth (positive, so bits order like values); once an
                         // uplift view's pairs are placed, the Gaussian's first pair index instead
  uint32_t live;         // reachable blocks among the first 32 of the box (see pair_live)
};
static_assert(sizeof(GSplat) == 48, "GSplat layout");

// Whether Gaussian g can reach alpha >= 1/255 at any pixel centre of block
// (bx, by) (edge 1 << shift pixels, clipped to the W x H image): the minimum
// of q over the rectangle of pixel centres is zero if the centre lies inside,
// else the smallest of the four edge minima (each a clamped 1D quadratic).
// Conservative: a block is dropped only if that minimum exceeds log2(255 o)
// by a relative 1e-4 (plus 1e-4), far beyond float32 rounding of either side.
// The per-Gaussian constants are set up once for all blocks of its box.
struct BlockCull {
  int ix, iy, shift, W, H;
  float fx, fy, a, b, c, rh, rv, thr;
  __device__ __forceinline__ BlockCull(const GSplat& g, int shift_, int W_, int H_) {
    ix = g.ix; iy = g.iy; fx = g.fx; fy = g.fy; shift = shift_; W = W_; H = H_;
    a = g.l00; b = g.l10; c = g.l11;
    rh = -b / a;                                   // horizontal edge: argmin dx = rh dy
    rv = -a * b / fmaf(b, b, c * c);               // vertical edge: argmin dy = rv dx
    thr = fmaf(log2f(255.0f * g.opacity), 1.0001f, 1e-4f);
  }
  __device__ __forceinline__ float q(float dx, float dy) const {
    const float u = fmaf(a, dx, b * dy), v = c * dy;
    return fmaf(u, u, v * v);
  }
  __device__ __forceinline__ bool live(int bx, int by) const {
    const int x_lo = bx << shift, y_lo = by << shift;
    return live_rect(x_lo, min(x_lo + (1 << shift), W) - 1, y_lo, min(y_lo + (1 << shift), H) - 1);
  }
  // the same test on the pixel rectangle [x_lo, x_hi] x [y_lo, y_hi] (inclusive)
  __device__ __forceinline__ bool live_rect(int x_lo, int x_hi, int y_lo, int y_hi) const {
    const float xa = ((float)(x_lo - ix) + 0.5f) - fx, xb = ((float)(x_hi - ix) + 0.5f) - fx;
    const float ya = ((float)(y_lo - iy) + 0.5f) - fy, yb = ((float)(y_hi - iy) + 0.5f) - fy;
    if (xa <= 0.0f && xb >= 0.0f && ya <= 0.0f && yb >= 0.0f) return true;
    const float h0 = q(fminf(fmaxf(rh * ya, xa), xb), ya);
    const float h1 = q(fminf(fmaxf(rh * yb, xa), xb), yb);
    const float v0 = q(xa, fminf(fmaxf(rv * xa, ya), yb));
    const float v1 = q(xb, fminf(fmaxf(rv * xb, ya), yb));
    return fminf(fminf(h0, h1), fminf(v0, v1)) <= thr;
  }
};

// Bit r of GSplat::live is set when block r (row-major in the Gaussian's
// block box) is reachable, for the first 32 blocks; later blocks are tested
// again where needed.
__device__ __forceinline__ bool pair_live(const GSplat& g, const BlockCull& bc, int r, int bx, int by) {
  return r < 32 ? ((g.live >> r) & 1u) != 0u : bc.live(bx, by);
}

// One batch Gaussian held by its lane, in block-relative form for the
// compositing loop: integer centre offset from the block origin (exact in
// float32), fraction, scaled conic factor, opacity and the largest q that
// still gives alpha >= 1/255 (alpha = o 2^-q >= 1/255  <=>  q <= log2(255 o)).
struct BlockSplat {
  float hx, hy, fx, fy, l00, l10, l11, opacity, qmax;
  __device__ __forceinline__ void load(const GSplat& g, int x0, int y0) {
    hx = (float)(g.ix - x0); hy = (float)(g.iy - y0);
    fx = g.fx; fy = g.fy; l00 = g.l00; l10 = g.l10; l11 = g.l11; opacity = g.opacity;
    qmax = g.opacity > 0.0f ? log2f(255.0f * g.opacity) : -1.0f;
  }
  __device__ __forceinline__ BlockSplat bcast(int k) const {
    BlockSplat r;
    r.hx = rl(hx, k); r.hy = rl(hy, k); r.fx = rl(fx, k); r.fy = rl(fy, k);
    r.l00 = rl(l00, k); r.l10 = rl(l10, k); r.l11 = rl(l11, k); r.opacity = rl(opacity, k); r.qmax = rl(qmax, k);
    return r;
  }
  static __device__ __forceinline__ float rl(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
  }
};

// Small per-call status block in the workspace.
struct Status {
  unsigned int total_pairs;     // pairs of the current view
  unsigned int view_overflow;   // current view exceeded the pair capacity
  unsigned int any_overflow;
  unsigned int max_pairs;       // largest per-view pair count seen
  unsigned int data_error;      // region id out of range
  unsigned int n_big;           // tiles of the current view sorted in global memory
  unsigned long long n_extra;   // deferred further-region entry slots reserved in the current view
  unsigned long long contrib;   // contributions composited
  unsigned long long touches;   // statistics: distinct (Gaussian, region) pairs with weight, level 0
  unsigned long long touch_lost;  // statistics: pairs the counting set could not place
  unsigned long long n_direct;  // further-region weights added straight to the accumulator
};

struct CamDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int width, height;
  float near_z;
};

// Sum over the 64 lanes of a wave, the same value returned to every lane.
// DPP within rows of 16 (xor 1, xor 2 via quad permutes, rotate 4 and 8),
// then the four row sums are read from lanes 0, 16, 32, 48 (fixed order).
template <int CTRL>
__device__ __forceinline__ float dpp_shuffle(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_shuffle<0xb1>(v);    // quad_perm [1,0,3,2]
  v += dpp_shuffle<0x4e>(v);    // quad_perm [2,3,0,1]
  v += dpp_shuffle<0x124>(v);   // row_ror:4
  v += dpp_shuffle<0x128>(v);   // row_ror:8
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

template <int CTRL>
__device__ __forceinline__ unsigned int dpp_u32(unsigned int v) {
  return (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ void max_step_u64(unsigned int& hi, unsigned int& lo) {
  const unsigned int h2 = dpp_u32<CTRL>(hi), l2 = dpp_u32<CTRL>(lo);
  const bool take = h2 > hi || (h2 == hi && l2 > lo);
  hi = take ? h2 : hi;
  lo = take ? l2 : lo;
}

// Maximum over the 64 lanes of a wave of a 64-bit key, returned to every lane.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  unsigned int hi = (unsigned int)(v >> 32), lo = (unsigned int)v;
  max_step_u64<0xb1>(hi, lo);
  max_step_u64<0x4e>(hi, lo);
  max_step_u64<0x124>(hi, lo);
  max_step_u64<0x128>(hi, lo);
  unsigned long long best = 0ull;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned int h = (unsigned int)__builtin_amdgcn_readlane((int)hi, 16 * r);
    const unsigned int l = (unsigned int)__builtin_amdgcn_readlane((int)lo, 16 * r);
    const unsigned long long k = ((unsigned long long)h << 32) | l;
    best = k > best ? k : best;
  }
  return best;
}

// float32 -> bfloat16, round to nearest even (a NaN stays a NaN): the
// hardware conversion (v_cvt_pk_bf16_f32), which on gfx950 rounds every
// non-NaN float32, subnormals and overflow to infinity included, exactly as
// adding 0x7fff plus the kept lowest bit and truncating does.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// two values, the first in the low half
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned int f32x2_to_bf16(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(unsigned int, __builtin_convertvector(v, bf16x2_t));
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((unsigned int)b << 16); }

// float32 -> OCP FP8 E4M3 (bias 7, 3 mantissa bits, max 448, no infinities),
// round to nearest even, saturating to +-448: the hardware conversion
// (v_cvt_pk_fp8_f32, round to nearest even, subnormals kept) of the value
// clamped to +-448 first, since larger magnitudes would convert to NaN.
__device__ __forceinline__ float e4m3_clamp(float x) { return x != x ? x : fminf(fmaxf(x, -448.0f), 448.0f); }

__device__ __forceinline__ uint8_t f32_to_e4m3(float x) {
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(x), 0.0f, 0, false) & 0xff);
}

// four values, the first in the low byte
__device__ __forceinline__ unsigned int f32x4_to_e4m3(float a, float b, float c, float d) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(a), e4m3_clamp(b), 0, false);
  return (unsigned int)__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(c), e4m3_clamp(d), lo, true);
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// bitonic sorting network, every comparator ascending (min to the lower
// index): positions past the end act as +infinity and are never touched.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cmp_swap(unsigned long long* a, unsigned long long* b) {
  const unsigned long long x = *a, y = *b;
  if (x > y) { *a = y; *b = x; }
}

__device__ inline void bitonic_lds(unsigned long long* s, int n2, int tid, int nthreads) {
  for (int k = 2; k <= n2; k <<= 1) {
    const int hk = k >> 1;
    for (int i = tid; i < (n2 >> 1); i += nthreads) {
      const int blk = i / hk, off = i - blk * hk;
      cmp_swap(&s[blk * k + off], &s[blk * k + k - 1 - off]);
    }
    __syncthreads();
    for (int j = k >> 2; j >= 1; j >>= 1) {
      for (int i = tid; i < (n2 >> 1); i += nthreads) {
        const int blk = i / j, off = i - blk * j;
        const int a = blk * 2 * j + off;
        cmp_swap(&s[a], &s[a + j]);
      }
      __syncthreads();
    }
  }
}

}  // namespace scoup
