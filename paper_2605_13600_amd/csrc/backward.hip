// Backward of render (Eq. 7) and decode (Eq. 8) for a loss L(F):
//   dL/dC          = W_hat^T G                 (k_gemm_at_b, float32 MFMA, split over pixels)
//   dL/dW_hat(p)   = G(p) C^T                  (the decode GEMM with a transposed codebook)
//   dL/dw_hat_i[k] = sum_{p} e_i(p) dL/dW_hat(p)[idx_ik]   (k_render_bwd)
// with G = dL/dF.  Atom indices and geometry receive no gradient.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

typedef float f16v __attribute__((ext_vector_type(16)));
constexpr int kBwdKMax = 16;

// One 8x8 pixel block per workgroup (one wave): recompute e = alpha T front to
// back, gather dL/dW_hat at each Gaussian's K atoms from the block's rows in
// LDS, reduce over the block's pixels and add to grad_val.
__global__ __launch_bounds__(64) void k_render_bwd(
    const GSplat* __restrict__ splats, const unsigned int* __restrict__ tile_start,
    const unsigned int* __restrict__ order,
    const unsigned long long* __restrict__ keys, int tiles_x, int W, int H,
    const int* __restrict__ topk_idx, int K, int M, const float* __restrict__ dW,
    float* __restrict__ grad_val, Status* st) {
  extern __shared__ float rows[];          // 64 * (M+1) floats
  __shared__ unsigned int s_id[64];
  __shared__ int s_ti[64 * kBwdKMax];
  if (st->view_overflow) return;
  const int tile = (int)order[blockIdx.x];      // longest lists first
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const unsigned int start = tile_start[tile];
  const int L = (int)(tile_start[tile + 1] - start);
  if (L == 0) return;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int tile_x0 = tx * 8, tile_y0 = ty * 8;
  const int px = tile_x0 + lx, py = tile_y0 + ly;
  const bool inside = px < W && py < H;
  const int stride = M + 1;

  for (int p = 0; p < 64; ++p) {
    const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
    const bool in = ox < W && oy < H;
    const float* src = dW + ((long long)oy * W + ox) * M;
    for (int j = lane; j < M; j += 64) rows[p * stride + j] = in ? src[j] : 0.0f;
  }
  __syncthreads();

  const float* myrow = rows + lane * stride;
  float T = inside ? 1.0f : -1.0f;             // transmittance, negated once the pixel is finished
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  for (int b0 = 0; b0 < L; b0 += 64) {
    if (__ballot(T > 0.0f) == 0ull) break;
    const int j = b0 + lane;
    BlockSplat mine;
    if (j < L) {
      const unsigned int id = (unsigned int)keys[start + j];
      mine.load(splats[id], tile_x0, tile_y0);
      s_id[lane] = id;
      for (int k = 0; k < K; ++k) s_ti[lane * K + k] = topk_idx[(long long)id * K + k];
    }
    __syncthreads();
    const int nb = min(64, L - b0);
    for (int k = 0; k < nb; ++k) {
      const BlockSplat g = mine.bcast(k);
      const float dx = (pcx - g.hx) - g.fx, dy = (pcy - g.hy) - g.fy;
      const float u = fmaf(g.l00, dx, g.l10 * dy), v = g.l11 * dy;
      const float q = fmaf(u, u, v * v);
      // branchless front-to-back step; T < 0 marks a finished pixel
      const float alpha = fminf(kAlphaMax, g.opacity * __builtin_amdgcn_exp2f(-q));
      const float testT = T * (1.0f - alpha);
      const bool take = T > 0.0f && q <= g.qmax;
      const bool keep = take && testT >= kTMin;
      const float e = keep ? alpha * T : 0.0f;
      T = take ? (keep ? testT : -T) : T;
      if (__ballot(keep)) {
        float gsum = 0.0f;
        for (int kk = 0; kk < K; ++kk) {
          const int jj = s_ti[k * K + kk];
          const float prod = (e > 0.0f && jj >= 0 && jj < M) ? e * myrow[jj] : 0.0f;
          const float sum = wave_sum(prod);
          if (lane == kk) gsum = sum;
        }
        if (lane < K && gsum != 0.0f) atomic_add_f32(&grad_val[(long long)s_id[k] * K + lane], gsum);
      }
      if (__ballot(T > 0.0f) == 0ull) break;
    }
    __syncthreads();
  }
}

// grad_C[m, d] += sum_p coeff[p, m] G[p, d]; workgroup tile 128 (m) x 128 (d)
// over one pixel chunk, 4 waves of 32 x 128; operands straight from global
// memory (each k-step reads two 128-byte rows per operand fragment).
__global__ __launch_bounds__(256) void k_gemm_at_b(const float* __restrict__ A, const float* __restrict__ G,
                                                   long long P, int M, int D, long long chunk,
                                                   float* __restrict__ out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.x * 128 + wave * 32;
  const int d0 = blockIdx.y * 128;
  const long long pb = (long long)blockIdx.z * chunk;
  const long long pe = min(P, pb + chunk);
  const int mi = m0 + (lane & 31);
  f16v acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = (f16v){};
  for (long long p = pb; p < pe; p += 2) {
    const long long pr = p + (lane >> 5);
    const bool okp = pr < pe;
    const float a = (okp && mi < M) ? A[pr * M + mi] : 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int dj = d0 + c * 32 + (lane & 31);
      const float b = (okp && dj < D) ? G[pr * D + dj] : 0.0f;
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int d = d0 + c * 32 + (lane & 31);
      if (m < M && d < D && acc[c][r] != 0.0f) atomic_add_f32(&out[(long long)m * D + d], acc[c][r]);
    }
}

hipError_t launch_gemm_at_b(const float* coeff, const float* G, long long P, int m, int d, float* grad_C,
                            hipStream_t s) {
  if (P == 0) return hipSuccess;
  const int mt = (m + 127) / 128, dt = (d + 127) / 128;
  long long nch = std::max(1, 1024 / (mt * dt));
  long long chunk = (P + nch - 1) / nch;
  chunk = (chunk + 1) & ~1ll;
  nch = (P + chunk - 1) / chunk;
  StageTimer::begin(kStBwdGemm, s);
  hipLaunchKernelGGL(k_gemm_at_b, dim3(mt, dt, (unsigned)nch), dim3(256), 0, s, coeff, G, P, m, d, chunk,
                     grad_C);
  StageTimer::end(kStBwdGemm, s);
  return hipGetLastError();
}

hipError_t launch_render_bwd_view(RenderBwdArgs& a, hipStream_t s) {
  hipError_t e = launch_bin_view(a.bin, s);
  if (e != hipSuccess) return e;
  const BinArgs& b = a.bin;
  const size_t lds = sizeof(float) * 64 * (size_t)(a.m_atoms + 1);
  StageTimer::begin(kStRenderBwd, s);
  hipLaunchKernelGGL(k_render_bwd, dim3(b.n_tiles), dim3(64), lds, s, b.splats, b.tile_start, b.tile_order, b.keys[b.sorted],
                     b.tiles_x, b.cam.width, b.cam.height, a.topk_idx, a.k, a.m_atoms, a.dW,
                     a.grad_val, b.status);
  StageTimer::end(kStRenderBwd, s);
  return hipGetLastError();
}

hipError_t render_bwd_set_lds_limits() {
  const int bytes = 160 * 1024 - (int)(sizeof(GSplat) * 64 + 4 * 64 + 4 * 64 * kBwdKMax) - 1024;
  return hipFuncSetAttribute((const void*)k_render_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace scoup
