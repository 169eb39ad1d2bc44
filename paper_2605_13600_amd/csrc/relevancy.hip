// Relevancy of rendered language features to text queries (App. B), fused with
// the codebook decode of Eq. 8.
//
// The score only needs the dot products of F(p) = W_hat(p) C with the query
// and canonical vectors t, and F(p).t = W_hat(p) (C t).  So the codebook is
// folded into the vectors once (S = C T, M x 32, in FP64) and the per-pixel
// work is a skinny [P x M] x [M x 32] contraction on MFMA followed by the
// score epilogue: the P x D feature map is never formed, and the kernel
// streams the coefficient map from HBM once.
//
// MFMA tile (operands swapped so that each lane owns one pixel): rows are 32
// "slots" of S^T, columns are 32 pixels.  Lane l holds slots
// 8 (r/4) + 4 (l/32) + r%4 for r = 0..15 of pixel l%32.  Slots 0-3 and 4-7
// both carry the (up to four) canonical vectors, one copy per lane half, and
// the other 24 slots carry queries, so every lane finds the canonical scores
// of its pixel in its own registers.  More than 24 queries run as further
// query groups (grid y).
//
// Precision: float32 coefficient maps use the float32 MFMA with S rounded to
// float32; bfloat16 and FP8 maps (FP8 converted exactly to bfloat16 in
// registers) use the bfloat16 MFMA with S split into a high and a low
// bfloat16 part, so S carries about 16 significant bits.
#include <hip/hip_runtime.h>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

constexpr int kRelWaves = 4;                 // waves per workgroup, each on its own pixels
constexpr int kRelTile = 64;                 // pixels per wave: two 32-column MFMA tiles
constexpr int kRelChunk = 128;               // bytes of every coefficient row staged per step
constexpr int kRelStride = kRelChunk + 16;   // LDS row stride (16-byte aligned, spreads banks)
constexpr int kRelPieces = kRelTile * kRelChunk / 16 / 64;   // 16-byte loads per lane per chunk

// Per input type: element size, MFMA k-step, k-steps per chunk and the bytes
// one lane reads from its row per k-step.  Lane half h of the tile covers
// the h-th 64-byte half of each chunk row, k-step kk the kk-th slice of it.
template <int T> struct RelT;
template <> struct RelT<SCOUP_F32> { static constexpr int ES = 4, KS = 2, KPC = 16, LB = 4; };
template <> struct RelT<SCOUP_BF16> { static constexpr int ES = 2, KS = 16, KPC = 4, LB = 16; };
template <> struct RelT<SCOUP_FP8_E4M3> { static constexpr int ES = 1, KS = 16, KPC = 8, LB = 8; };

// Slot s of a query group: s / 8 == 0 is canonical vector s % 4; otherwise
// query 4 (2 (s/8 - 1) + (s/4) % 2) + s % 4 of the group.
__host__ __device__ __forceinline__ int rel_query_of_slot(int s) {
  return 4 * (2 * (s / 8 - 1) + (s / 4) % 2) + (s % 4);
}

// S fragment element (group g, slot s, atom m): position in the A-operand
// fragment array of the MFMA (units of elements), k permuted as described.
template <int T>
__device__ __forceinline__ long long rel_frag_pos(int g, int nks, int s, int m) {
  using R = RelT<T>;
  constexpr int CE = kRelChunk / R::ES;      // elements per chunk row
  constexpr int H = R::KS / 2;               // elements per lane per k-step
  const int ch = m / CE, r = m % CE;
  const int h = r / (CE / 2), r2 = r % (CE / 2);
  const int kk = r2 / H, i = r2 % H;
  const int ks = ch * R::KPC + kk;
  const int lane = s + 32 * h;
  return (((long long)g * nks + ks) * 64 + lane) * H + i;
}

// S = C T in FP64: one thread per (group, slot, atom), atoms padded with zeros.
template <int T>
__global__ __launch_bounds__(256) void k_rel_prep(const float* __restrict__ C, int M, int D, int kpad,
                                                  int nks, int n_groups, const float* __restrict__ queries,
                                                  int Q, const float* __restrict__ canon, int n_canon,
                                                  void* __restrict__ frag, long long lo_off) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)n_groups * 32 * kpad;
  if (t >= total) return;
  const int m = (int)(t % kpad);
  const int s = (int)((t / kpad) % 32);
  const int g = (int)(t / ((long long)kpad * 32));
  const float* vec = nullptr;
  if (s < 8) {
    if (s % 4 < n_canon) vec = canon + (long long)(s % 4) * D;
  } else {
    const int q = g * 24 + rel_query_of_slot(s);
    if (q < Q) vec = queries + (long long)q * D;
  }
  double dot = 0.0;
  if (vec && m < M) {
    const float* row = C + (long long)m * D;
    if ((D & 3) == 0 && ((reinterpret_cast<uintptr_t>(C) | reinterpret_cast<uintptr_t>(vec)) & 15) == 0) {
      for (int d = 0; d < D; d += 4) {
        const float4 a = *reinterpret_cast<const float4*>(row + d);
        const float4 b = *reinterpret_cast<const float4*>(vec + d);
        dot = fma((double)a.x, (double)b.x, dot);
        dot = fma((double)a.y, (double)b.y, dot);
        dot = fma((double)a.z, (double)b.z, dot);
        dot = fma((double)a.w, (double)b.w, dot);
      }
    } else {
      for (int d = 0; d < D; ++d) dot = fma((double)row[d], (double)vec[d], dot);
    }
  }
  const long long pos = rel_frag_pos<T>(g, nks, s, m);
  if (T == SCOUP_F32) {
    reinterpret_cast<float*>(frag)[pos] = (float)dot;
  } else {
    const uint16_t hi = f32_to_bf16_rne((float)dot);
    const uint16_t lo = f32_to_bf16_rne((float)(dot - (double)bf16_to_f32(hi)));
    reinterpret_cast<uint16_t*>(frag)[pos] = hi;
    reinterpret_cast<uint16_t*>(frag)[lo_off + pos] = lo;
  }
}

// exact OCP E4M3 -> bfloat16 (every E4M3 value is a bfloat16 value): the
// hardware decodes a byte pair to float32 (v_cvt_pk_f32_fp8), the exact
// narrowing to bfloat16 packs the pair again
__device__ __forceinline__ bf16x8 e4m3x8_to_bf16(i32x2 v) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  i32x4 o;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const f2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(v[w], false);
    const f2 hi = __builtin_amdgcn_cvt_pk_f32_fp8(v[w], true);
    o[2 * w] = (int)f32x2_to_bf16(lo[0], lo[1]);
    o[2 * w + 1] = (int)f32x2_to_bf16(hi[0], hi[1]);
  }
  return __builtin_bit_cast(bf16x8, o);
}

// LDS traffic of one wave stays inside its own region: order the wave's own
// writes before its reads (and reads before the next chunk's writes).
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <int T>
__global__ __launch_bounds__(kRelWaves * 64) void k_relevancy(
    const uint8_t* __restrict__ A, long long P, int row_bytes, int nchunks, int nks,
    const uint8_t* __restrict__ frag, long long lo_off, int n_canon, int Q, float out_mul, float temp,
    float* __restrict__ out, int vec_in, int vec_out) {
  using R = RelT<T>;
  __shared__ i32x4 s_rows[kRelWaves][kRelTile * kRelStride / 16];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long p0 = ((long long)blockIdx.x * kRelWaves + wave) * kRelTile;
  if (p0 >= P) return;                       // wave-uniform; no workgroup barrier below
  const int g = blockIdx.y;
  uint8_t* rows = reinterpret_cast<uint8_t*>(s_rows[wave]);
  const bool aligned = vec_in != 0;           // rows and base 16-byte aligned
  const int h = lane >> 5, n = lane & 31;

  // chunk ch of the tile's rows, 16 bytes per lane per piece, zero past the row and past P
  auto load_chunk = [&](int ch, i32x4* v) {
#pragma unroll
    for (int i = 0; i < kRelPieces; ++i) {
      const int piece = i * 64 + lane;
      const int r = piece >> 3, q = piece & 7;
      const long long p = p0 + r;
      const int off = ch * kRelChunk + q * 16;
      i32x4 x = {0, 0, 0, 0};
      if (p < P && off < row_bytes) {
        const uint8_t* src = A + p * row_bytes + off;
        if (aligned) {
          x = __builtin_nontemporal_load(reinterpret_cast<const i32x4*>(src));
        } else {                             // rows not 16-byte aligned: assemble bytewise
#pragma unroll
          for (int b = 0; b < 16; ++b)
            if (off + b < row_bytes) x[b >> 2] |= (int)src[b] << (8 * (b & 3));
        }
      }
      v[i] = x;
    }
  };

  f16v acc[2] = {(f16v){}, (f16v){}};
  i32x4 buf[kRelPieces];
  load_chunk(0, buf);
  for (int ch = 0; ch < nchunks; ++ch) {
#pragma unroll
    for (int i = 0; i < kRelPieces; ++i) {
      const int piece = i * 64 + lane;
      *reinterpret_cast<i32x4*>(rows + (piece >> 3) * kRelStride + (piece & 7) * 16) = buf[i];
    }
    wave_lds_sync();
    // this lane's 64-byte half of rows n and 32 + n
    i32x4 b0[4], b1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      b0[j] = *reinterpret_cast<const i32x4*>(rows + n * kRelStride + h * 64 + j * 16);
      b1[j] = *reinterpret_cast<const i32x4*>(rows + (32 + n) * kRelStride + h * 64 + j * 16);
    }
    wave_lds_sync();
    if (ch + 1 < nchunks) load_chunk(ch + 1, buf);
#pragma unroll
    for (int kk = 0; kk < R::KPC; ++kk) {
      const int ks = ch * R::KPC + kk;
      const long long fi = ((long long)g * nks + ks) * 64 + lane;
      if constexpr (T == SCOUP_F32) {
        const float a = reinterpret_cast<const float*>(frag)[fi];
        const float w0 = __int_as_float(b0[kk / 4][kk % 4]);
        const float w1 = __int_as_float(b1[kk / 4][kk % 4]);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, w0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, w1, acc[1], 0, 0, 0);
      } else {
        const bf16x8 ahi = reinterpret_cast<const bf16x8*>(frag)[fi];
        const bf16x8 alo = reinterpret_cast<const bf16x8*>(frag + lo_off * 2)[fi];
        bf16x8 w0, w1;
        if constexpr (T == SCOUP_BF16) {
          w0 = __builtin_bit_cast(bf16x8, b0[kk]);
          w1 = __builtin_bit_cast(bf16x8, b1[kk]);
        } else {
          const i32x2 x0 = {b0[kk / 2][2 * (kk % 2)], b0[kk / 2][2 * (kk % 2) + 1]};
          const i32x2 x1 = {b1[kk / 2][2 * (kk % 2)], b1[kk / 2][2 * (kk % 2) + 1]};
          w0 = e4m3x8_to_bf16(x0);
          w1 = e4m3x8_to_bf16(x1);
        }
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, w0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, w1, acc[1], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, w0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, w1, acc[1], 0, 0, 0);
      }
    }
  }

  // epilogue: R = min_k sigma(a (s_q - s_ck)) = sigma(a (s_q - max_k s_ck))
  const bool vec = vec_out != 0;              // Q % 4 == 0 and out 16-byte aligned
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const long long p = p0 + t * 32 + n;
    if (p >= P) continue;
    float cmax = acc[t][0] * out_mul;
#pragma unroll
    for (int j = 1; j < 4; ++j)
      if (j < n_canon) cmax = fmaxf(cmax, acc[t][j] * out_mul);
    float* orow = out + p * Q;
#pragma unroll
    for (int rg = 1; rg < 4; ++rg) {
      const int q0 = g * 24 + 4 * (2 * (rg - 1) + h);
      float r[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) r[j] = 1.0f / (1.0f + expf(temp * (cmax - acc[t][4 * rg + j] * out_mul)));
      if (vec && q0 + 3 < Q) {
        *reinterpret_cast<float4*>(orow + q0) = make_float4(r[0], r[1], r[2], r[3]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (q0 + j < Q) orow[q0 + j] = r[j];
      }
    }
  }
}

static int rel_es(int in_dtype) { return in_dtype == SCOUP_F32 ? 4 : in_dtype == SCOUP_BF16 ? 2 : 1; }

int relevancy_groups(int q) { return (q + 23) / 24; }

static int rel_nchunks(int m, int in_dtype) { return (m * rel_es(in_dtype) + kRelChunk - 1) / kRelChunk; }

static int rel_nks(int m, int in_dtype) {
  const int kpc = in_dtype == SCOUP_F32 ? 16 : in_dtype == SCOUP_BF16 ? 4 : 8;
  return rel_nchunks(m, in_dtype) * kpc;
}

// elements of one S fragment array (the bfloat16 types hold two: high and low)
static long long rel_frag_elems(int m, int q, int in_dtype) {
  const int half = in_dtype == SCOUP_F32 ? 1 : 8;
  return (long long)relevancy_groups(q) * rel_nks(m, in_dtype) * 64 * half;
}

size_t relevancy_frag_bytes(int m, int q, int in_dtype) {
  const long long e = rel_frag_elems(m, q, in_dtype);
  return in_dtype == SCOUP_F32 ? (size_t)e * 4 : (size_t)e * 2 * 2;
}

hipError_t launch_relevancy(const RelevancyArgs& a, hipStream_t s) {
  const int ng = relevancy_groups(a.Q);
  const int nchunks = rel_nchunks(a.m, a.in_dtype);
  const int nks = rel_nks(a.m, a.in_dtype);
  const int kpad = nchunks * (kRelChunk / rel_es(a.in_dtype));
  const long long lo_off = rel_frag_elems(a.m, a.Q, a.in_dtype);
  const long long prep_threads = (long long)ng * 32 * kpad;
  const int pgrid = (int)((prep_threads + 255) / 256);
  StageTimer::begin(kStRelPrep, s);
  switch (a.in_dtype) {
    case SCOUP_F32:
      hipLaunchKernelGGL(k_rel_prep<SCOUP_F32>, dim3(pgrid), dim3(256), 0, s, a.codebook, a.m, a.d, kpad, nks, ng,
                         a.queries, a.Q, a.canon, a.n_canon, a.frag, lo_off);
      break;
    case SCOUP_BF16:
      hipLaunchKernelGGL(k_rel_prep<SCOUP_BF16>, dim3(pgrid), dim3(256), 0, s, a.codebook, a.m, a.d, kpad, nks,
                         ng, a.queries, a.Q, a.canon, a.n_canon, a.frag, lo_off);
      break;
    default:
      hipLaunchKernelGGL(k_rel_prep<SCOUP_FP8_E4M3>, dim3(pgrid), dim3(256), 0, s, a.codebook, a.m, a.d, kpad,
                         nks, ng, a.queries, a.Q, a.canon, a.n_canon, a.frag, lo_off);
      break;
  }
  StageTimer::end(kStRelPrep, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  StageTimer::begin(kStRelevancy, s);
  const long long tiles = (a.P + kRelTile - 1) / kRelTile;
  const dim3 grid((unsigned int)((tiles + kRelWaves - 1) / kRelWaves), (unsigned int)ng);
  if (tiles > 0) {
    const int rb = a.m * rel_es(a.in_dtype);
    const uint8_t* A = static_cast<const uint8_t*>(a.coeff);
    const uint8_t* F = static_cast<const uint8_t*>(a.frag);
    const int vin = (rb % 16 == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0);
    const int vout = (a.Q % 4 == 0) && (reinterpret_cast<uintptr_t>(a.out) % 16 == 0);
    switch (a.in_dtype) {
      case SCOUP_F32:
        hipLaunchKernelGGL(k_relevancy<SCOUP_F32>, grid, dim3(kRelWaves * 64), 0, s, A, a.P, rb, nchunks, nks, F,
                           lo_off, a.n_canon, a.Q, a.out_mul, a.temperature, a.out, vin, vout);
        break;
      case SCOUP_BF16:
        hipLaunchKernelGGL(k_relevancy<SCOUP_BF16>, grid, dim3(kRelWaves * 64), 0, s, A, a.P, rb, nchunks, nks,
                           F, lo_off, a.n_canon, a.Q, a.out_mul, a.temperature, a.out, vin, vout);
        break;
      default:
        hipLaunchKernelGGL(k_relevancy<SCOUP_FP8_E4M3>, grid, dim3(kRelWaves * 64), 0, s, A, a.P, rb, nchunks,
                           nks, F, lo_off, a.n_canon, a.Q, a.out_mul, a.temperature, a.out, vin, vout);
        break;
    }
  }
  StageTimer::end(kStRelevancy, s);
  return hipGetLastError();
}

}  // namespace scoup
