// Backward of render (Eq. 7) and decode (Eq. 8) for a loss L(F):
//   dL/dC          = W_hat^T G                 (k_gemm_at_b per pixel chunk + k_sum_parts)
//   dL/dW_hat(p)   = G(p) C^T                  (the decode GEMM with a transposed codebook)
//   dL/dw_hat_i[k] = sum_{p} e_i(p) dL/dW_hat(p)[idx_ik]   (k_render_bwd per (Gaussian, block)
//                                                           + k_pair_reduce)
// with G = dL/dF.  Atom indices and geometry receive no gradient.
//
// Every sum has a fixed order, so the gradients are deterministic: the GEMM
// writes one partial product per pixel chunk and a second kernel adds the
// chunks in chunk order; the render backward writes one partial per
// (Gaussian, 8x8 block) pair into the pair's slot (Gaussian-major, the
// binning's pair offsets) and a per-Gaussian kernel adds its pairs in box
// order.  Only those two final kernels write the caller's gradients, and both
// do nothing when the view's pair count exceeded the capacity, so a failed
// call leaves them untouched.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

typedef float f16v __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// dL/dC partial products: part[c][m][d] = sum over the pixels p of chunk c of
// A[p][m] G[p][d].  Workgroup tile 128 (m) x 128 (d), four waves of 32 x 128
// (four 32x32 float32 MFMA accumulators each); 16-pixel stages of both
// operands are loaded with 16-byte loads into registers one stage ahead, then
// stored to LDS (double buffered), and each k-step (two pixels) reads its
// MFMA fragments from LDS.
// ---------------------------------------------------------------------------
constexpr int kGemmStage = 16;

template <bool VEC>
__device__ __forceinline__ float4 load_row4(const float* __restrict__ base, long long p, long long pe, int ld,
                                            int c) {
  float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (p >= pe) return r;
  const float* src = base + p * (long long)ld + c;
  if (VEC) {
    if (c < ld) r = *reinterpret_cast<const float4*>(src);
  } else {
    if (c + 0 < ld) r.x = src[0];
    if (c + 1 < ld) r.y = src[1];
    if (c + 2 < ld) r.z = src[2];
    if (c + 3 < ld) r.w = src[3];
  }
  return r;
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_gemm_at_b(const float* __restrict__ A, const float* __restrict__ G,
                                                   long long P, int M, int D, long long chunk,
                                                   float* __restrict__ part) {
  __shared__ float sA[2][kGemmStage][128];
  __shared__ float sG[2][kGemmStage][128];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.x * 128, d0 = blockIdx.y * 128;
  const long long pb = (long long)blockIdx.z * chunk;
  const long long pe = min(P, pb + chunk);
  // staging: thread t holds rows (t >> 5) and (t >> 5) + 8 of the stage, columns 4 (t & 31) .. +3
  const int sr = tid >> 5, sc = 4 * (tid & 31);
  float4 ra[2], rg[2];
  auto load = [&](long long p0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      ra[h] = load_row4<VEC>(A, p0 + sr + 8 * h, pe, M, m0 + sc);
      rg[h] = load_row4<VEC>(G, p0 + sr + 8 * h, pe, D, d0 + sc);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<float4*>(&sA[buf][sr + 8 * h][sc]) = ra[h];
      *reinterpret_cast<float4*>(&sG[buf][sr + 8 * h][sc]) = rg[h];
    }
  };
  f16v acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = (f16v){};
  if (pb < pe) {
    load(pb);
    store(0);
    __syncthreads();
    int buf = 0;
    for (long long p0 = pb; p0 < pe; p0 += kGemmStage) {
      const bool more = p0 + kGemmStage < pe;
      if (more) load(p0 + kGemmStage);
      // lane l supplies row (l & 31) at k = l >> 5 of A^T and column (l & 31) at k = l >> 5 of G
#pragma unroll
      for (int s = 0; s < kGemmStage / 2; ++s) {
        const int pr = 2 * s + (lane >> 5);
        const float a = sA[buf][pr][32 * wave + (lane & 31)];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float b = sG[buf][pr][32 * c + (lane & 31)];
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
        }
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  float* out = part + (long long)blockIdx.z * M * D;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + 32 * wave + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int d = d0 + 32 * c + (lane & 31);
      if (m < M && d < D) out[(long long)m * D + d] = acc[c][r];
    }
}

// out[e] += sum_c part[c][e], chunks in order (nothing on a failed view)
__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ part, int nch, long long n,
                                                   float* __restrict__ out, const Status* st) {
  if (st->any_overflow) return;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float s = 0.0f;
  for (int c = 0; c < nch; ++c) s += part[(long long)c * n + e];
  out[e] += s;
}

int gemm_at_b_chunks(long long P, int m, int d) {
  const int tiles = ((m + 127) / 128) * ((d + 127) / 128);
  long long nch = std::max(1, kGemmMaxParts / tiles);
  nch = std::min<long long>(nch, (P + 4 * kGemmStage - 1) / (4 * kGemmStage));   // at least 64 pixels each
  return (int)std::max<long long>(1, nch);
}

hipError_t launch_gemm_at_b(const float* coeff, const float* G, long long P, int m, int d, float* part,
                            float* grad_C, const Status* st, hipStream_t s) {
  int nch = gemm_at_b_chunks(P, m, d);
  long long chunk = (P + nch - 1) / nch;
  chunk = (chunk + kGemmStage - 1) / kGemmStage * kGemmStage;
  nch = (int)std::max<long long>(1, (P + chunk - 1) / chunk);
  const dim3 grid((m + 127) / 128, (d + 127) / 128, nch);
  const bool vec = (m & 3) == 0 && (d & 3) == 0 &&
                   ((reinterpret_cast<uintptr_t>(coeff) | reinterpret_cast<uintptr_t>(G)) & 15) == 0;
  StageTimer::begin(kStBwdGemm, s);
  if (P > 0) {
    if (vec)
      hipLaunchKernelGGL(k_gemm_at_b<true>, grid, dim3(256), 0, s, coeff, G, P, m, d, chunk, part);
    else
      hipLaunchKernelGGL(k_gemm_at_b<false>, grid, dim3(256), 0, s, coeff, G, P, m, d, chunk, part);
    const long long n = (long long)m * d;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nch, n, grad_C, st);
  }
  StageTimer::end(kStBwdGemm, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dL/dw_hat per (Gaussian, 8x8 block): one wave per block.  The block's rows
// of dL/dW_hat (64 pixels x M, float32) sit in LDS.  Per batch of 32
// Gaussians of the block's depth-ordered list, the lanes (one per pixel)
// recompute e = alpha T front to back (the forward's arithmetic) into an LDS
// matrix E[Gaussian][pixel]; then lane (g, k) of each group of 64 / K
// contributing Gaussians forms sum_p E[g][p] dW[p][idx_gk] (four partial sums
// over p mod 4, added in a fixed order) and writes it to the pair's slot.
// ---------------------------------------------------------------------------
constexpr int kBwdBatch = 32;            // two blocks' LDS fit a CU at M = 256

__global__ __launch_bounds__(64) void k_render_bwd(
    const GSplat* __restrict__ splats, const unsigned int* __restrict__ tile_start,
    const unsigned int* __restrict__ order,
    const unsigned long long* __restrict__ keys, int tiles_x, int W, int H,
    const int* __restrict__ topk_idx, int K, int M, const float* __restrict__ dW,
    float* __restrict__ pair_part, const Status* st) {
  extern __shared__ float rows[];          // 64 * (M+1) floats
  __shared__ float sE[kBwdBatch][65];      // E[g][p], rows padded against bank conflicts
  __shared__ int s_ti[kBwdBatch * kBwdKMax];
  __shared__ unsigned int s_slot[kBwdBatch];
  __shared__ unsigned char s_live[kBwdBatch];
  if (st->any_overflow) return;
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

  float T = inside ? 1.0f : -1.0f;             // transmittance, negated once the pixel is finished
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  const int gper = 64 / K;                     // Gaussians per reduction pass
  const int rg = lane / K, rk = lane - (lane / K) * K;
  for (int b0 = 0; b0 < L; b0 += kBwdBatch) {
    if (__ballot(T > 0.0f) == 0ull) break;
    const int nb = min(kBwdBatch, L - b0);
    BlockSplat mine;
    if (lane < nb) {
      const unsigned int id = (unsigned int)keys[start + b0 + lane];
      const GSplat sp = splats[id];
      mine.load(sp, tile_x0, tile_y0);
      // pair slot: the Gaussian's first pair (left in its splat by the binning)
      // + this block's row-major index in the Gaussian's block box
      const int bx0 = sp.bx0 >> 3, bx1 = sp.bx1 >> 3, by0 = sp.by0 >> 3;
      s_slot[lane] = sp.depth_bits + (unsigned int)((ty - by0) * (bx1 - bx0 + 1) + (tx - bx0));
      for (int k = 0; k < K; ++k) s_ti[lane * K + k] = topk_idx[(long long)id * K + k];
    }
    unsigned long long live = 0ull;            // Gaussians of the batch with a contribution
    int k = 0;
    for (; k < nb; ++k) {
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
      sE[k][lane] = e;
      if (__ballot(keep)) live |= 1ull << k;
      if (__ballot(T > 0.0f) == 0ull) { ++k; break; }
    }
    __syncthreads();                           // E, slots and indices of the batch are in LDS
    // contributing Gaussians, gper at a time: lane (rg, rk) reduces Gaussian rg's slot rk
    while (live) {
      int gi = -1;
      unsigned long long rest = live;
      for (int t = 0; t < gper && rest; ++t) {
        const int g = __ffsll((long long)rest) - 1;
        rest &= rest - 1ull;
        if (t == rg) gi = g;
      }
      live = rest;
      if (gi >= 0 && rk < K) {
        const int j = s_ti[gi * K + rk];
        if (j >= 0 && j < M) {
          float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
          const float* ep = sE[gi];
          const float* rp = rows + j;
#pragma unroll 4
          for (int p = 0; p < 64; p += 4) {
            s0 = fmaf(ep[p + 0], rp[(p + 0) * stride], s0);
            s1 = fmaf(ep[p + 1], rp[(p + 1) * stride], s1);
            s2 = fmaf(ep[p + 2], rp[(p + 2) * stride], s2);
            s3 = fmaf(ep[p + 3], rp[(p + 3) * stride], s3);
          }
          pair_part[(long long)s_slot[gi] * K + rk] = (s0 + s1) + (s2 + s3);
        }
      }
    }
    __syncthreads();                           // before the next batch overwrites E
  }
}

// pair_part[e] = 0 for the view's pairs (slots of pairs never composited stay zero)
__global__ __launch_bounds__(256) void k_clear_pairs(float* __restrict__ pair_part, int K, const Status* st) {
  if (st->any_overflow) return;
  const unsigned long long n = (unsigned long long)st->total_pairs * (unsigned long long)K;
  for (unsigned long long e = blockIdx.x * 256ull + threadIdx.x; e < n; e += gridDim.x * 256ull)
    pair_part[e] = 0.0f;
}

// grad_val[i][k] += sum over Gaussian i's pairs (box order) of pair_part[pair][k]
__global__ __launch_bounds__(256) void k_pair_reduce(const float* __restrict__ pair_part,
                                                     const unsigned int* __restrict__ offsets, long long n, int K,
                                                     float* __restrict__ grad_val, const Status* st) {
  if (st->any_overflow) return;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n * K) return;
  const long long i = t / K;
  const int k = (int)(t - i * K);
  const unsigned int b0 = offsets[i], b1 = offsets[i + 1];
  float s = 0.0f;
  for (unsigned int b = b0; b < b1; ++b) s += pair_part[(long long)b * K + k];
  if (b1 > b0) grad_val[t] += s;
}

hipError_t launch_render_bwd_view(RenderBwdArgs& a, hipStream_t s) {
  const BinArgs& b = a.bin;
  const size_t lds = sizeof(float) * 64 * (size_t)(a.m_atoms + 1);
  StageTimer::begin(kStRenderBwd, s);
  hipLaunchKernelGGL(k_clear_pairs, dim3(1024), dim3(256), 0, s, a.pair_part, a.k, (const Status*)b.status);
  hipLaunchKernelGGL(k_render_bwd, dim3(b.n_tiles), dim3(64), lds, s, b.splats, b.tile_start, b.tile_order,
                     b.keys[b.sorted], b.tiles_x, b.cam.width, b.cam.height, a.topk_idx, a.k, a.m_atoms, a.dW,
                     a.pair_part, (const Status*)b.status);
  if (b.n > 0)
    hipLaunchKernelGGL(k_pair_reduce, dim3((unsigned)((b.n * a.k + 255) / 256)), dim3(256), 0, s, a.pair_part,
                       (const unsigned int*)b.offsets, b.n, a.k, a.grad_val, (const Status*)b.status);
  StageTimer::end(kStRenderBwd, s);
  return hipGetLastError();
}

hipError_t render_bwd_set_lds_limits() {
  const int bytes = 160 * 1024 - (int)(4 * kBwdBatch * 65 + 4 * kBwdBatch * kBwdKMax + 5 * kBwdBatch) - 1024;
  return hipFuncSetAttribute((const void*)k_render_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace scoup
