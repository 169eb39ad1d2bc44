// Sparse coefficient render (Eq. 7): W_hat_v(p) = sum_{i in N_{v,p}} w_hat_i e_i(v,p)
// over K (atom, value) pairs per Gaussian, front-to-back weights e from Eq. 2.
// gfx950, wave64: one 8x8 pixel block per workgroup (one wave), its list in
// depth order (binning); every pixel
// keeps its dense M-wide coefficient row in LDS (stride M+1 to spread banks),
// accumulates in float32 and writes the row once, converted to the output type.
#include <hip/hip_runtime.h>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

constexpr int kRenderKMax = 16;

__device__ __forceinline__ void store_out(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_out(uint16_t* p, float v) { *p = f32_to_bf16_rne(v); }
__device__ __forceinline__ void store_out(uint8_t* p, float v) { *p = f32_to_e4m3(v); }

// Four waves per 8x8 block share its LDS rows: wave w composites pixel rows
// 2w and 2w+1 (16 pixels, lane & 15), and the four lane groups of 16 (lane >> 4)
// each add every fourth code slot of a contributing Gaussian.  The front-to-
// back recurrence is evaluated by all four lane groups of a pixel (no cross-lane
// traffic); what the split buys is four waves in flight per block instead of one,
// since the block's 64 KB of rows allow only two blocks per CU.
constexpr int kRenderWaves = 4;
constexpr int kRenderBatch = 16;          // Gaussians staged per wave and batch

// order of one wave's own LDS writes before its reads (and reads before rewrites)
__device__ __forceinline__ void render_wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <typename OutT>
__global__ __launch_bounds__(64 * kRenderWaves) void k_render_coeff(
    const GSplat* __restrict__ splats, const unsigned int* __restrict__ tile_start,
    const unsigned int* __restrict__ order,
    const unsigned long long* __restrict__ keys, int tiles_x, int W, int H,
    const int* __restrict__ topk_idx, const float* __restrict__ topk_val, int K, int M,
    OutT* __restrict__ out, float out_scale, float* __restrict__ t_final, Status* st) {
  extern __shared__ float rows[];          // 64 * (M+1) floats
  __shared__ int s_ti[kRenderWaves][kRenderBatch * kRenderKMax];
  __shared__ float s_tv[kRenderWaves][kRenderBatch * kRenderKMax];
  if (st->view_overflow) return;
  const int tile = (int)order[blockIdx.x];      // longest lists first
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const unsigned int start = tile_start[tile];
  const int L = (int)(tile_start[tile + 1] - start);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int pix = wave * 16 + (lane & 15), sub = lane >> 4;
  const int lx = pix & 7, ly = pix >> 3;
  const int tile_x0 = tx * 8, tile_y0 = ty * 8;
  const int px = tile_x0 + lx, py = tile_y0 + ly;
  const bool inside = px < W && py < H;
  const int stride = M + 1;

  for (int j = tid; j < 64 * stride; j += 64 * kRenderWaves) rows[j] = 0.0f;
  __syncthreads();

  float* myrow = rows + pix * stride;
  int* ti = s_ti[wave];
  float* tv = s_tv[wave];
  float T = inside ? 1.0f : -1.0f;             // transmittance, negated once the pixel is finished
  unsigned int count = 0u;
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  // The batch's ids arrive two batches ahead, its splats and code slots one
  // batch ahead (registers), so no batch waits on a dependent load chain;
  // indices past the list are clamped to its last entry (loads unconditional).
  // Lane l holds Gaussian l & 15 of a batch; code slot t = l + 64 i of the
  // batch is slot t % K of Gaussian t / K.
  constexpr int TK = (kRenderBatch * kRenderKMax + 63) / 64;
  const int kb = lane & (kRenderBatch - 1);
  const int nslots = kRenderBatch * K;
  auto key_at = [&](int i) { return (unsigned int)keys[start + min(i, L - 1)]; };
  auto load_codes = [&](unsigned int keyv, int (&ci)[TK], float (&cv)[TK]) {
#pragma unroll
    for (int i = 0; i < TK; ++i) {
      const int t = min(lane + 64 * i, nslots - 1);
      const int k = t / K, j = t - k * K;
      const unsigned int id = (unsigned int)__shfl((int)keyv, k, 64);
      ci[i] = topk_idx[(long long)id * K + j];
      cv[i] = topk_val[(long long)id * K + j];
    }
  };
  if (L > 0) {
    unsigned int key_c = key_at(kb), key_n = key_at(kRenderBatch + kb);
    GSplat sp_c = splats[key_c];
    int ci_c[TK];
    float cv_c[TK];
    load_codes(key_c, ci_c, cv_c);
    for (int b0 = 0; b0 < L; b0 += kRenderBatch) {
      if (__ballot(T > 0.0f) == 0ull) break;
      const int nb = min(kRenderBatch, L - b0);
      const GSplat sp_n = splats[key_n];
      int ci_n[TK];
      float cv_n[TK];
      load_codes(key_n, ci_n, cv_n);
      const unsigned int key_nn = key_at(b0 + 2 * kRenderBatch + kb);
      BlockSplat mine;
      bool reach = false;                      // Gaussian `lane` reaches this wave's two pixel rows
      if (lane < nb) {
        mine.load(sp_c, tile_x0, tile_y0);
        const BlockCull bc(sp_c, 3, W, H);
        const int ry = tile_y0 + 2 * wave;
        reach = ry < H && bc.live_rect(tile_x0, min(tile_x0 + 8, W) - 1, ry, min(ry + 2, H) - 1);
      }
      unsigned long long queue = __ballot(reach);
#pragma unroll
      for (int i = 0; i < TK; ++i) {
        const int t = lane + 64 * i;
        if (t < nb * K) { ti[t] = ci_c[i]; tv[t] = cv_c[i]; }
      }
      render_wave_lds_sync();
      while (queue) {                          // only the batch Gaussians that reach these rows
        const int k = __ffsll((long long)queue) - 1;
        queue &= queue - 1ull;
        const BlockSplat g = mine.bcast(k);
        const float dx = (pcx - g.hx) - g.fx, dy = (pcy - g.hy) - g.fy;
        const float u = fmaf(g.l00, dx, g.l10 * dy), v = g.l11 * dy;
        const float q = fmaf(u, u, v * v);
        // branchless front-to-back step; a finished pixel keeps -T (its final transmittance, negated)
        const float alpha = fminf(kAlphaMax, g.opacity * __builtin_amdgcn_exp2f(-q));
        const float testT = T * (1.0f - alpha);
        const bool take = T > 0.0f && q <= g.qmax;
        const bool keep = take && testT >= kTMin;
        const float e = keep ? alpha * T : 0.0f;
        T = take ? (keep ? testT : -T) : T;
        if (keep) {
          count += sub == 0 ? 1u : 0u;
          for (int kk = sub; kk < K; kk += 4) {   // fire-and-forget LDS adds: no read-modify-write chain
            const int jj = ti[k * K + kk];
            if (jj >= 0 && jj < M) atomicAdd(&myrow[jj], e * tv[k * K + kk]);
            else if (jj >= M) atomicOr(&st->data_error, 4u);
          }
        }
        if (__ballot(T > 0.0f) == 0ull) break;
      }
      render_wave_lds_sync();
      key_c = key_n;
      key_n = key_nn;
      sp_c = sp_n;
#pragma unroll
      for (int i = 0; i < TK; ++i) { ci_c[i] = ci_n[i]; cv_c[i] = cv_n[i]; }
    }
  }
  if (inside && sub == 0 && t_final) t_final[(long long)py * W + px] = fabsf(T);
  unsigned long long total = count;
  for (int o = 32; o >= 1; o >>= 1) total += __shfl_xor(total, o, 64);
  if (lane == 0 && total) atomicAdd(&st->contrib, total);
  // this wave's 16 pixel rows are complete (its own LDS adds are ordered before
  // these reads); write them, atoms fastest (coalesced per pixel row)
  render_wave_lds_sync();
  for (int p = wave * 16; p < wave * 16 + 16; ++p) {
    const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
    if (ox >= W || oy >= H) continue;
    OutT* dst = out + ((long long)oy * W + ox) * M;
    const float* src = rows + p * stride;
    for (int jj = lane; jj < M; jj += 64) store_out(dst + jj, src[jj] * out_scale);
  }
}

hipError_t launch_render_view(RenderViewArgs& a, hipStream_t s) {
  hipError_t e = launch_bin_view(a.bin, s);
  if (e != hipSuccess) return e;
  const BinArgs& b = a.bin;
  const size_t lds = sizeof(float) * 64 * (size_t)(a.m_atoms + 1);
  StageTimer::begin(kStRender, s);
  switch (a.out_dtype) {
    case SCOUP_F32:
      hipLaunchKernelGGL(k_render_coeff<float>, dim3(b.n_tiles), dim3(64 * kRenderWaves), lds, s, b.splats, b.tile_start,
                         b.tile_order, b.keys[b.sorted], b.tiles_x, b.cam.width, b.cam.height, a.topk_idx, a.topk_val, a.k,
                         a.m_atoms, (float*)a.out, a.out_scale, a.t_final, b.status);
      break;
    case SCOUP_BF16:
      hipLaunchKernelGGL(k_render_coeff<uint16_t>, dim3(b.n_tiles), dim3(64 * kRenderWaves), lds, s, b.splats,
                         b.tile_start, b.tile_order, b.keys[b.sorted], b.tiles_x, b.cam.width, b.cam.height, a.topk_idx,
                         a.topk_val, a.k, a.m_atoms, (uint16_t*)a.out, a.out_scale,
                         a.t_final, b.status);
      break;
    default:
      hipLaunchKernelGGL(k_render_coeff<uint8_t>, dim3(b.n_tiles), dim3(64 * kRenderWaves), lds, s, b.splats,
                         b.tile_start, b.tile_order, b.keys[b.sorted], b.tiles_x, b.cam.width, b.cam.height, a.topk_idx,
                         a.topk_val, a.k, a.m_atoms, (uint8_t*)a.out, a.out_scale,
                         a.t_final, b.status);
      break;
  }
  StageTimer::end(kStRender, s);
  return hipGetLastError();
}

hipError_t render_set_lds_limits() {
  const int bytes = 160 * 1024 - (int)(8 * kRenderWaves * kRenderBatch * kRenderKMax) - 1024;
  hipError_t e = hipFuncSetAttribute((const void*)k_render_coeff<float>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_render_coeff<uint16_t>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_render_coeff<uint8_t>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             bytes);
}

}  // namespace scoup
