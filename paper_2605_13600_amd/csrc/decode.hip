// Codebook decode (Eq. 8): F = W_hat C, [P x M] x [M x D], on MFMA with float32
// accumulation.  Input precisions: float32 (v_mfma_f32_32x32x2_f32),
// bfloat16 (v_mfma_f32_32x32x16_bf16) and OCP FP8 E4M3 with power-of-two
// per-tensor scales (v_mfma_scale_f32_32x32x64_f8f6f4, unit block scales).
// Output float32 or bfloat16.
//
// Workgroup: 8 waves, one 128-pixel x D tile at a time (one workgroup per CU
// walks the tiles).  The 128 x M coefficient rows are staged in LDS, each
// thread issuing its 16-byte row loads together; the codebook is pre-arranged
// in MFMA B-fragment order (one 1 KB coalesced load per 32-column tile and
// k-step) and read from L2.  Wave w owns pixels [64 (w/4), +64) and columns
// [(w%4) D/4, +D/4).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// k-step and fragment bytes per lane of each input type
template <int T> struct Mfma;
template <> struct Mfma<SCOUP_F32> { static constexpr int KS = 2, FB = 4, ES = 4; };
template <> struct Mfma<SCOUP_BF16> { static constexpr int KS = 16, FB = 16, ES = 2; };
template <> struct Mfma<SCOUP_FP8_E4M3> { static constexpr int KS = 64, FB = 32, ES = 1; };

// operand fragment of one lane and the matching MFMA
template <int T> struct Frag;
template <> struct Frag<SCOUP_F32> {
  typedef float type;
  static __device__ __forceinline__ f16v mfma(float a, float b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Frag<SCOUP_BF16> {
  typedef bf16x8 type;
  static __device__ __forceinline__ f16v mfma(bf16x8 a, bf16x8 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Frag<SCOUP_FP8_E4M3> {
  typedef i32x8 type;
  // format 0 = FP8 E4M3 for both operands; E8M0 block scales 127 = 2^0
  static __device__ __forceinline__ f16v mfma(i32x8 a, i32x8 b, f16v c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
};

constexpr int kDecBM = 128;
constexpr int kDecThreads = 512;
constexpr int kDecGrid = 256;                 // one workgroup per CU (registers allow one)

// lane l of a 32x32 MFMA operand covers row/col (l % 32) and the k-slice
// [(l / 32) * KS/2, +KS/2) of the k-step.
// B operand (K x N = M x D here) from a float32 source, element (k, n) at
// C[k * N + n] (or C[n * K + k] when transposed); columns beyond N are zero.
template <int T>
__global__ __launch_bounds__(256) void k_prep_codebook(const float* __restrict__ C, int M, int D, int kpad,
                                                       int npad, int transposed, uint8_t* __restrict__ out,
                                                       const float* scale_ptr) {
  using F = Mfma<T>;
  const long long total = (long long)(npad / 32) * (kpad / F::KS) * 64;   // (ct, ks, lane)
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int lane = (int)(t & 63);
  const long long rest = t >> 6;
  const int nks = kpad / F::KS;
  const int ks = (int)(rest % nks), ct = (int)(rest / nks);
  const int col = ct * 32 + (lane & 31);
  const int k0 = ks * F::KS + (lane >> 5) * (F::KS / 2);
  const float sc = scale_ptr ? *scale_ptr : 1.0f;
  uint8_t* dst = out + t * F::FB;
  for (int i = 0; i < F::KS / 2; ++i) {
    const int k = k0 + i;
    const float v = (k < M && col < D)
                        ? (transposed ? C[(long long)col * M + k] : C[(long long)k * D + col]) * sc
                        : 0.0f;
    if (T == SCOUP_F32) reinterpret_cast<float*>(dst)[i] = v;
    else if (T == SCOUP_BF16) reinterpret_cast<uint16_t*>(dst)[i] = f32_to_bf16_rne(v);
    else dst[i] = f32_to_e4m3(v);
  }
}

// max |C| as float bits (non-negative floats order like their bit patterns)
__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ C, long long n,
                                                unsigned int* __restrict__ maxbits) {
  __shared__ float red[256];
  float m = 0.0f;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    m = fmaxf(m, fabsf(C[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(maxbits, __float_as_uint(red[0]));
}

// power-of-two scale s with max|C| s <= 448 (FP8 E4M3 range)
__device__ __forceinline__ float fp8_scale_from(unsigned int maxbits) {
  const float mx = __uint_as_float(maxbits);
  return mx > 0.0f ? exp2f(floorf(log2f(448.0f / mx))) : 1.0f;
}

__global__ void k_clear_u32(unsigned int* p) { *p = 0u; }

__global__ void k_fp8_scale(const unsigned int* __restrict__ maxbits, float* scale) {
  scale[0] = fp8_scale_from(*maxbits);
}

__device__ __forceinline__ void store_f(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_f(uint16_t* p, float v) { *p = f32_to_bf16_rne(v); }
// four consecutive outputs (16-byte aligned float32 / 8-byte aligned bfloat16)
__device__ __forceinline__ void store4(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ void store4(uint16_t* p, float a, float b, float c, float d) {
  const unsigned int lo = f32x2_to_bf16(a, b);
  const unsigned int hi = f32x2_to_bf16(c, d);
  *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi);
}

template <int T, int NCT, typename TOut>
__global__ __launch_bounds__(kDecThreads) void k_decode(const uint8_t* __restrict__ A, long long P, int M,
                                                        int kpad, int kc, const uint8_t* __restrict__ Bp,
                                                        int n_valid, int ldo, TOut* __restrict__ out,
                                                        float out_mul, const float* __restrict__ cb_scale,
                                                        int staged_out, int ct_base) {
  using F = Mfma<T>;
  using FT = typename Frag<T>::type;
  extern __shared__ uint8_t sA[];                     // kDecBM rows of kc elements (+16 B pad)
  const int row_bytes = kc * F::ES + 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int src_row = M * F::ES;
  const int rh = wave >> 2, cq = wave & 3;
  const int nks = kpad / F::KS;
  const int ct0 = ct_base + cq * NCT;             // the launch covers column tiles ct_base .. + 4 NCT - 1
  const long long n_tiles = (P + kDecBM - 1) / kDecBM;
  float mul = out_mul;
  if (cb_scale) mul /= *cb_scale;
  // workgroups walk tiles blockIdx.x, + gridDim.x, ...
  constexpr int U = 8;                         // 16-byte row pieces a thread loads before storing them
  // rows [p0, p0+128) x k [k0, k0+kcur) in 16-byte chunks, zero beyond M and P
  auto stage_chunk = [&](long long p0, int k0, int kcur) {
    const int chunks = kcur * F::ES / 16;
    const int total = kDecBM * chunks;
    if ((src_row & 15) == 0) {
      for (int c0 = tid; c0 < total; c0 += kDecThreads * U) {
        i32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int c = c0 + u * kDecThreads;
          const int r = c / chunks, q = c - r * chunks;
          const int off = k0 * F::ES + q * 16;
          v[u] = (i32x4){0, 0, 0, 0};
          if (c < total && p0 + r < P && off + 16 <= src_row)
            v[u] = *reinterpret_cast<const i32x4*>(A + (p0 + r) * src_row + off);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int c = c0 + u * kDecThreads;
          const int r = c / chunks, q = c - r * chunks;
          if (c < total) *reinterpret_cast<i32x4*>(sA + r * row_bytes + q * 16) = v[u];
        }
      }
    } else {
      for (int c = tid; c < total; c += kDecThreads) {
        const int r = c / chunks, q = c - r * chunks;
        i32x4 v = {0, 0, 0, 0};
        const long long p = p0 + r;
        const int off = k0 * F::ES + q * 16;
        if (p < P) {
          const uint8_t* src = A + p * src_row + off;
          unsigned int w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int b = 0; b < 16; ++b)
            if (off + b < src_row) w[b >> 2] |= (unsigned int)src[b] << (8 * (b & 3));
          v = (i32x4){(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
        }
        *reinterpret_cast<i32x4*>(sA + r * row_bytes + q * 16) = v;
      }
    }
  };
  // the MFMAs of k [k0, k0+kcur) from LDS for column tiles cb .. cb + NC - 1 of
  // the wave (acc is f16v[2][NC]); codebook fragments one k-step ahead
  auto mfma_cols = [&](int k0, int kcur, int cb, auto& acc) {
    constexpr int NC = (int)(sizeof(acc[0]) / sizeof(f16v));
    FT bcur[NC], bnext[NC];
    const FT* Bf = reinterpret_cast<const FT*>(Bp);
#pragma unroll
    for (int c = 0; c < NC; ++c) bcur[c] = Bf[((long long)(cb + c) * nks + k0 / F::KS) * 64 + lane];
    const int ks_last = (k0 + kcur) / F::KS - 1;
    for (int kk = 0; kk < kcur; kk += F::KS) {
      const int ks = (k0 + kk) / F::KS;
      // unconditional (the last step reloads its own fragment): a fixed count
      // of loads per step lets each multiply wait for its own fragment only
      const int ksn = min(ks + 1, ks_last);
#pragma unroll
      for (int c = 0; c < NC; ++c) bnext[c] = Bf[((long long)(cb + c) * nks + ksn) * 64 + lane];
      const int kb = (kk + (lane >> 5) * (F::KS / 2)) * F::ES;   // byte offset in the LDS row
      const FT a0 = *reinterpret_cast<const FT*>(sA + (rh * 64 + (lane & 31)) * row_bytes + kb);
      const FT a1 = *reinterpret_cast<const FT*>(sA + (rh * 64 + 32 + (lane & 31)) * row_bytes + kb);
      // operands swapped: the tile is F^T = C^T W^T, so each lane owns one pixel
      // and runs of four consecutive feature columns (vector stores below)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[0][c] = Frag<T>::mfma(bcur[c], a0, acc[0][c]);
        acc[1][c] = Frag<T>::mfma(bcur[c], a1, acc[1][c]);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) bcur[c] = bnext[c];
    }
  };
  // element (row 8(r/4) + 4(l/32) + r%4, col l%32) of each 32x32 tile of F^T:
  // pixel p0 + rh*64 + a*32 + l%32, feature column (cb+c)*32 + 8(r/4) + 4(l/32) + r%4
  auto epilogue = [&](long long p0, int cb, const auto& acc) {
    constexpr int NC = (int)(sizeof(acc[0]) / sizeof(f16v));
    const bool vec = (ldo & 3) == 0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const long long p = p0 + rh * 64 + a * 32 + (lane & 31);
      if (p >= P) continue;
      TOut* orow = out + p * ldo;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
          const int d0 = (cb + c) * 32 + 8 * rg + 4 * (lane >> 5);
          const float v0 = acc[a][c][4 * rg] * mul, v1 = acc[a][c][4 * rg + 1] * mul;
          const float v2 = acc[a][c][4 * rg + 2] * mul, v3 = acc[a][c][4 * rg + 3] * mul;
          if (vec && d0 + 3 < n_valid) {
            store4(orow + d0, v0, v1, v2, v3);
          } else {
            if (d0 < n_valid) store_f(orow + d0, v0);
            if (d0 + 1 < n_valid) store_f(orow + d0 + 1, v1);
            if (d0 + 2 < n_valid) store_f(orow + d0 + 2, v2);
            if (d0 + 3 < n_valid) store_f(orow + d0 + 3, v3);
          }
        }
    }
  };

  for (long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const long long p0 = tile * kDecBM;
    f16v acc[2][NCT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < NCT; ++c) acc[a][c] = (f16v){};
    for (int k0 = 0; k0 < kpad; k0 += kc) {
      const int kcur = min(kc, kpad - k0);
      stage_chunk(p0, k0, kcur);
      __syncthreads();
      mfma_cols(k0, kcur, ct0, acc);
      __syncthreads();
    }
    if (staged_out) {
      // 32 pixels at a time: the waves holding them write their rows into LDS
      // (free after the k loop), then all threads store whole rows, 16 bytes a lane
      constexpr int OES = (int)sizeof(TOut);
      constexpr int OSTRIDE = 128 * NCT * OES + 16;
      const int col0 = ct_base * 32;               // the launch's first feature column
      const int cpr = min(128 * NCT, n_valid - col0) * OES / 16;
#pragma unroll
      for (int grp = 0; grp < 4; ++grp) {      // unrolled: acc[grp & 1] stays in registers
        if (rh == (grp >> 1)) {
          const int a = grp & 1;
          TOut* row = reinterpret_cast<TOut*>(sA + (lane & 31) * OSTRIDE);
#pragma unroll
          for (int c = 0; c < NCT; ++c)
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
              const int d0 = (cq * NCT + c) * 32 + 8 * rg + 4 * (lane >> 5);   // column within the launch
              store4(row + d0, acc[a][c][4 * rg] * mul, acc[a][c][4 * rg + 1] * mul, acc[a][c][4 * rg + 2] * mul,
                     acc[a][c][4 * rg + 3] * mul);
            }
        }
        __syncthreads();
        for (int c = tid; c < 32 * cpr; c += kDecThreads) {
          const int r = c / cpr, q = c - r * cpr;
          const long long p = p0 + grp * 32 + r;
          if (p < P)
            *reinterpret_cast<i32x4*>(reinterpret_cast<uint8_t*>(out) + (p * (long long)ldo + col0) * OES + q * 16) =
                *reinterpret_cast<const i32x4*>(sA + r * OSTRIDE + q * 16);
        }
        __syncthreads();
      }
    } else {
      epilogue(p0, ct0, acc);
    }
  }
}

// ---------------------------------------------------------------------------
// Codebook-stationary decode (BF16 / FP8 input, D <= 512, BF16 M <= 256, FP8
// M <= 512): wave w holds the B fragments of column tile w for every k-step
// in registers for the whole launch, so the codebook is read once per wave
// instead of once per pixel tile.  Tiles of 64 pixels stream through a
// double-buffered LDS block: the next tile's rows are loaded into registers
// when a tile starts and reach LDS after its multiplies, so the tile's work
// hides their latency.  Each 32-pixel half of the output goes through
// its own LDS staging area (one shared area when two do not fit) and leaves
// as 16-byte pieces of whole rows; with two areas no barrier waits for the
// stores.  The k loop has a compile-time length NKS >= the k-steps (padding
// steps multiply zero rows by a zero codebook fragment), so it is
// straight-line code with constant LDS offsets.
// ---------------------------------------------------------------------------
constexpr int kBsRows = 64;                   // pixels per tile
// k-steps held in registers: 64 registers of codebook fragments (BF16: M <= 256; FP8: M <= 512)
template <int T> struct BsKs { static constexpr int N = T == SCOUP_BF16 ? 16 : 8; };

// the k loop's compile-time length: the k-steps rounded up to a quarter, a
// half or all of the register budget n; the staged rows span that many
// k-steps (zero past kpad)
__host__ __device__ constexpr int bs_nks(int nks, int n) { return nks <= n / 4 ? n / 4 : nks <= n / 2 ? n / 2 : n; }
__host__ __device__ constexpr int bs_row_bytes(int kfull, int es) { return kfull * es + 16; }
__host__ __device__ inline int bs_stage_stride(int d, int oes) { return ((d * oes + 15) & ~15) + 16; }
// staging areas: two when they fit beside the double-buffered tile
__host__ __device__ inline int bs_n_stage(int kpad, int es, int d, int oes) {
  return 2 * (size_t)kBsRows * bs_row_bytes(kpad, es) + 2 * 32 * (size_t)bs_stage_stride(d, oes) <= 160 * 1024 ? 2
                                                                                                          : 1;
}

template <int T, typename TOut, int NKS>
__global__ __launch_bounds__(1024) void k_decode_bs(const uint8_t* __restrict__ A, long long P, int M, int kpad,
                                                    const uint8_t* __restrict__ Bp, int n_valid, int ldo,
                                                    TOut* __restrict__ out, float out_mul,
                                                    const float* __restrict__ cb_scale) {
  using F = Mfma<T>;
  using FT = typename Frag<T>::type;
  extern __shared__ __align__(16) uint8_t lds[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nks = kpad / F::KS;                       // 1 <= nks <= NKS
  constexpr int rb = bs_row_bytes(NKS * F::KS, F::ES);
  uint8_t* sA0 = lds;
  uint8_t* sA1 = lds + (size_t)kBsRows * rb;
  constexpr int OES = (int)sizeof(TOut);
  const int sstride = bs_stage_stride(n_valid, OES);
  const int nst = bs_n_stage(NKS * F::KS, F::ES, n_valid, OES);
  uint8_t* stage0 = lds + 2 * (size_t)kBsRows * rb;
  float mul = out_mul;
  if (cb_scale) mul /= *cb_scale;
  // the wave's codebook column tile, every k-step (zero past nks), complete
  // before the loop so that no multiply waits on memory
  FT bf[NKS];
  {
    const FT* Bf = reinterpret_cast<const FT*>(Bp);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) bf[ks] = Bf[((long long)wave * nks + min(ks, nks - 1)) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
      if (ks >= nks) bf[ks] = FT{};
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);                 // vmcnt(0)
  const long long n_tiles = (P + kBsRows - 1) / kBsRows;
  const int src_row = M * F::ES;
  const int chunks = kpad * F::ES / 16;              // 16-byte pieces per staged row
  const int per_tile = kBsRows * chunks;
  const bool vec_src = (src_row & 15) == 0;
  // a thread's pieces of tile t: c = tid + u nthreads
  const int nthr = blockDim.x;
  auto load_piece = [&](long long t, int c) -> i32x4 {
    i32x4 v = {0, 0, 0, 0};
    const int r = c / chunks, q = c - r * chunks;
    const long long p = t * kBsRows + r;
    const int off = q * 16;
    if (c < per_tile && p < P) {
      const uint8_t* src = A + p * src_row + off;
      if (vec_src) {
        if (off + 16 <= src_row) v = *reinterpret_cast<const i32x4*>(src);
      } else {
        unsigned int w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int b = 0; b < 16; ++b)
          if (off + b < src_row) w[b >> 2] |= (unsigned int)src[b] << (8 * (b & 3));
        v = (i32x4){(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
      }
    }
    return v;
  };
  auto put_piece = [&](uint8_t* sA, int c, i32x4 v) {
    if (c < per_tile) {
      const int r = c / chunks, q = c - r * chunks;
      *reinterpret_cast<i32x4*>(sA + r * rb + q * 16) = v;
    }
  };
  constexpr int U = 2;                                // pieces a thread loads ahead (a BF16 M = 256 tile at 1024 threads)
  {                                                   // the rows' k padding, both buffers: zero for good
    const int pc = (NKS * F::KS - kpad) * F::ES / 16;
    for (int c = tid; c < 2 * kBsRows * pc; c += nthr) {
      const int r = c / pc, q = c - r * pc;
      *reinterpret_cast<i32x4*>(lds + (size_t)r * rb + kpad * F::ES + q * 16) = (i32x4){0, 0, 0, 0};
    }
  }
  long long t = blockIdx.x;
  if (t < n_tiles) {
    for (int c0 = tid; c0 < per_tile; c0 += nthr * U) {
      i32x4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = load_piece(t, c0 + u * nthr);
#pragma unroll
      for (int u = 0; u < U; ++u) put_piece(sA0, c0 + u * nthr, v[u]);
    }
  }
  __syncthreads();
  const int rbytes = n_valid * OES;
  const bool vec = (rbytes & 15) == 0 && (((long long)ldo * OES) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  uint8_t* ob = reinterpret_cast<uint8_t*>(out);
  int buf = 0;
  for (; t < n_tiles; t += gridDim.x) {
    uint8_t* sA = buf ? sA1 : sA0;
    uint8_t* sN = buf ? sA0 : sA1;
    const long long tn = t + gridDim.x;
    // the next tile's rows: loads issued now, stored after the multiplies
    i32x4 nv[U];
    const bool more = tn < n_tiles && per_tile <= nthr * U;
#pragma unroll
    for (int u = 0; u < U; ++u) nv[u] = more ? load_piece(tn, tid + u * nthr) : (i32x4){0, 0, 0, 0};
    // element r of lane l: pixel h 32 + l % 32, feature 32 wave + 8 (r / 4) + 4 (l / 32) + r % 4
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f16v acc = (f16v){};
      const uint8_t* arow = sA + (h * 32 + (lane & 31)) * rb + (lane >> 5) * (F::KS / 2) * F::ES;
      if constexpr (T == SCOUP_FP8_E4M3 && NKS == BsKs<T>::N) {
        // one k-step per branch: straight-line code would let the scheduler
        // hoist every 8-register FP8 operand ahead of the multiplies and spill
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks)
          if (ks < nks) acc = Frag<T>::mfma(bf[ks], *reinterpret_cast<const FT*>(arow + ks * F::KS * F::ES), acc);
      } else {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks)
          acc = Frag<T>::mfma(bf[ks], *reinterpret_cast<const FT*>(arow + ks * F::KS * F::ES), acc);
      }
      if (h == 1 && more) {
        // the next tile's rows into the other buffer (its last reader, the
        // previous tile's multiplies, is behind the previous barriers; the
        // next tile reads it after the barrier below)
#pragma unroll
        for (int u = 0; u < U; ++u) put_piece(sN, tid + u * nthr, nv[u]);
      }
      uint8_t* stage = stage0 + (nst == 2 ? h : 0) * 32 * (size_t)sstride;
      TOut* row = reinterpret_cast<TOut*>(stage + (lane & 31) * sstride);
#pragma unroll
      for (int rg = 0; rg < 4; ++rg) {
        const int d0 = wave * 32 + 8 * rg + 4 * (lane >> 5);
        if (d0 + 3 < n_valid) {
          store4(row + d0, acc[4 * rg] * mul, acc[4 * rg + 1] * mul, acc[4 * rg + 2] * mul, acc[4 * rg + 3] * mul);
        } else {
          if (d0 < n_valid) store_f(row + d0, acc[4 * rg] * mul);
          if (d0 + 1 < n_valid) store_f(row + d0 + 1, acc[4 * rg + 1] * mul);
          if (d0 + 2 < n_valid) store_f(row + d0 + 2, acc[4 * rg + 2] * mul);
        }
      }
      __syncthreads();
      const long long p0 = t * kBsRows + h * 32;
      if (vec) {
        const int pieces = rbytes / 16;
        for (int c = tid; c < 32 * pieces; c += nthr) {
          const int r = c / pieces, q = c - r * pieces;
          if (p0 + r < P)
            *reinterpret_cast<i32x4*>(ob + (p0 + r) * (long long)ldo * OES + q * 16) =
                *reinterpret_cast<const i32x4*>(stage + r * sstride + q * 16);
        }
      } else {
        for (int c = tid; c < 32 * rbytes; c += nthr) {
          const int r = c / rbytes, b = c - r * rbytes;
          if (p0 + r < P) ob[(p0 + r) * (long long)ldo * OES + b] = stage[r * sstride + b];
        }
      }
      // one shared staging area: read out before the next half writes it.
      // Two: the next writer of this one is a half away, behind its barrier
      if (nst == 1) __syncthreads();
    }
    if (!more && tn < n_tiles) {                     // rows longer than one pass of loads
      for (int c0 = tid; c0 < per_tile; c0 += nthr * U) {
        i32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load_piece(tn, c0 + u * nthr);
#pragma unroll
        for (int u = 0; u < U; ++u) put_piece(sN, c0 + u * nthr, v[u]);
      }
      __syncthreads();
    }
    buf ^= 1;
  }
}

size_t decode_bs_lds_bytes(const DecodeArgs& a) {
  const int es = a.in_dtype == SCOUP_BF16 ? 2 : 1;
  const int oes = a.out_dtype == SCOUP_F32 ? 4 : 2;
  const int ks = a.in_dtype == SCOUP_BF16 ? 16 : 64;
  const int n = a.in_dtype == SCOUP_BF16 ? BsKs<SCOUP_BF16>::N : BsKs<SCOUP_FP8_E4M3>::N;
  const int kfull = bs_nks(a.kpad / ks, n) * ks;
  return 2 * (size_t)kBsRows * bs_row_bytes(kfull, es) +
         bs_n_stage(kfull, es, a.d, oes) * 32 * (size_t)bs_stage_stride(a.d, oes);
}

// BF16 / FP8 input, at most 16 column tiles and kBsMaxKs k-steps, LDS within 160 KB
bool decode_uses_bs(const DecodeArgs& a) {
  if (a.in_dtype != SCOUP_BF16 && a.in_dtype != SCOUP_FP8_E4M3) return false;
  const int ks = a.in_dtype == SCOUP_BF16 ? 16 : 64;
  const int maxks = a.in_dtype == SCOUP_BF16 ? BsKs<SCOUP_BF16>::N : BsKs<SCOUP_FP8_E4M3>::N;
  return decode_npad(a.d) <= 512 && a.kpad / ks <= maxks && decode_bs_lds_bytes(a) <= 160 * 1024;
}

int decode_npad(int d) {
  if (d <= 128) return 128;
  if (d <= 256) return 256;
  if (d <= 512) return 512;
  return 1024;
}

// K is padded (with zeros) to a multiple of both the MFMA k-step and one
// 16-byte LDS chunk: 4 (float32), 16 (bfloat16), 64 (FP8).
int decode_kalign(int in_dtype) { return in_dtype == SCOUP_F32 ? 4 : in_dtype == SCOUP_BF16 ? 16 : 64; }

int decode_kpad(int m, int in_dtype) {
  const int ka = decode_kalign(in_dtype);
  return (m + ka - 1) / ka * ka;
}

size_t decode_codebook_bytes(int m, int d, int in_dtype) {
  const int es = in_dtype == SCOUP_F32 ? 4 : in_dtype == SCOUP_BF16 ? 2 : 1;
  return (size_t)decode_kpad(m, in_dtype) * decode_npad(d) * es;
}

// k-chunk staged in LDS per pass: at most 128 KB of coefficient rows
int decode_kchunk(int m, int in_dtype) {
  const int es = in_dtype == SCOUP_F32 ? 4 : in_dtype == SCOUP_BF16 ? 2 : 1;
  const int kpad = decode_kpad(m, in_dtype);
  const int cap = (128 * 1024 / kDecBM - 16) / es;         // elements per row
  const int ka = decode_kalign(in_dtype);
  const int kc = cap / ka * ka;
  return kpad < kc ? kpad : kc;
}

size_t decode_lds_bytes(int m, int in_dtype) {
  const int es = in_dtype == SCOUP_F32 ? 4 : in_dtype == SCOUP_BF16 ? 2 : 1;
  return (size_t)kDecBM * (decode_kchunk(m, in_dtype) * es + 16);
}

// Output rows staged through LDS and stored 16 bytes a lane (rows starting and
// ending on 16-byte boundaries; the workgroup's LDS then covers 32 staged
// rows): measured faster for float32 input (MFMA-bound, long k loop), slower
// for BF16 / FP8 input, whose short k loop leaves the barriers exposed.
template <int NCT, typename TOut>
static bool decode_staged_out(const DecodeArgs& a) {
  const int oes = (int)sizeof(TOut), ldo = a.ldo > 0 ? a.ldo : a.d;
  return a.in_dtype == SCOUP_F32 && (reinterpret_cast<uintptr_t>(a.out) & 15) == 0 &&
         ((long long)ldo * oes) % 16 == 0 && (a.d * oes) % 16 == 0;
}

template <int T, int NCT, typename TOut>
static void launch_dec(const DecodeArgs& a, hipStream_t s, size_t lds, int grid, int ct_base = 0) {
  const bool staged = decode_staged_out<NCT, TOut>(a);
  if (staged) lds = std::max(lds, (size_t)32 * (128 * NCT * sizeof(TOut) + 16));
  hipLaunchKernelGGL((k_decode<T, NCT, TOut>), dim3(grid), dim3(kDecThreads), lds, s,
                     (const uint8_t*)a.coeff, a.P, a.m, a.kpad, decode_kchunk(a.m, a.in_dtype),
                     (const uint8_t*)a.codebook_prep, a.d, a.ldo > 0 ? a.ldo : a.d, (TOut*)a.out, a.out_mul,
                     a.cb_scale, staged ? 1 : 0, ct_base);
}

template <int T, typename TOut>
static hipError_t dispatch_nct(const DecodeArgs& a, hipStream_t s, size_t lds, int grid) {
  switch (decode_npad(a.d) / 128) {
    case 1: launch_dec<T, 1, TOut>(a, s, lds, grid); break;
    case 2: launch_dec<T, 2, TOut>(a, s, lds, grid); break;
    case 4: launch_dec<T, 4, TOut>(a, s, lds, grid); break;
    case 8:                                   // 1024 columns: two launches of 512 (eight column
      launch_dec<T, 4, TOut>(a, s, lds, grid, 0);   // tiles a wave would spill their registers)
      launch_dec<T, 4, TOut>(a, s, lds, grid, 16);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int T, int NCT, typename TOut>
static hipError_t set_lds(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_decode<T, NCT, TOut>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int T, typename TOut>
static void launch_bs(const DecodeArgs& a, int g, int nw, size_t bl, int ldo, hipStream_t s) {
  constexpr int N = BsKs<T>::N;
  const int nks = a.kpad / Mfma<T>::KS;
#define BS_LAUNCH(NK)                                                                                            \
  hipLaunchKernelGGL((k_decode_bs<T, TOut, NK>), dim3(g), dim3(64 * nw), bl, s, (const uint8_t*)a.coeff, a.P, a.m, \
                     a.kpad, (const uint8_t*)a.codebook_prep, a.d, ldo, (TOut*)a.out, a.out_mul, a.cb_scale)
  switch (bs_nks(nks, N)) {
    case N / 4: BS_LAUNCH(N / 4); break;
    case N / 2: BS_LAUNCH(N / 2); break;
    default: BS_LAUNCH(N); break;
  }
#undef BS_LAUNCH
}

template <int T, typename TOut>
static hipError_t set_bs_lds(int b) {
  constexpr int N = BsKs<T>::N;
  const auto attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_decode_bs<T, TOut, N / 4>, attr, b)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_decode_bs<T, TOut, N / 2>, attr, b)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_decode_bs<T, TOut, N>, attr, b);
}

hipError_t decode_set_lds_limits() {
  const size_t b = 160 * 1024;
  hipError_t e = hipSuccess;
#define SETL(T, TO)                                                        \
  if ((e = set_lds<T, 1, TO>(b)) != hipSuccess) return e;                 \
  if ((e = set_lds<T, 2, TO>(b)) != hipSuccess) return e;                 \
  if ((e = set_lds<T, 4, TO>(b)) != hipSuccess) return e;
  SETL(SCOUP_F32, float) SETL(SCOUP_F32, uint16_t) SETL(SCOUP_BF16, float) SETL(SCOUP_BF16, uint16_t)
  SETL(SCOUP_FP8_E4M3, float) SETL(SCOUP_FP8_E4M3, uint16_t)
#undef SETL
  if ((e = set_bs_lds<SCOUP_BF16, float>((int)b)) != hipSuccess) return e;
  if ((e = set_bs_lds<SCOUP_BF16, uint16_t>((int)b)) != hipSuccess) return e;
  if ((e = set_bs_lds<SCOUP_FP8_E4M3, float>((int)b)) != hipSuccess) return e;
  return set_bs_lds<SCOUP_FP8_E4M3, uint16_t>((int)b);
}

hipError_t launch_prep_codebook(const float* C, int m, int d, int in_dtype, void* out, float* scale,
                                hipStream_t s, int transposed) {
  const int kpad = decode_kpad(m, in_dtype);
  const int npad = decode_npad(d);
  const int ks = in_dtype == SCOUP_F32 ? 2 : in_dtype == SCOUP_BF16 ? 16 : 64;
  const long long total = (long long)(npad / 32) * (kpad / ks) * 64;
  const int grid = (int)((total + 255) / 256);
  if (in_dtype == SCOUP_FP8_E4M3) {
    unsigned int* maxbits = reinterpret_cast<unsigned int*>(scale + 1);
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(1), 0, s, maxbits);   // a kernel, not a memset node
    const long long n = (long long)m * d;
    const int gb = (int)std::min<long long>(256, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax, dim3(gb), dim3(256), 0, s, C, n, maxbits);
    hipLaunchKernelGGL(k_fp8_scale, dim3(1), dim3(1), 0, s, (const unsigned int*)maxbits, scale);
    hipLaunchKernelGGL(k_prep_codebook<SCOUP_FP8_E4M3>, dim3(grid), dim3(256), 0, s, C, m, d, kpad, npad,
                       transposed, (uint8_t*)out, (const float*)scale);
  } else if (in_dtype == SCOUP_BF16) {
    hipLaunchKernelGGL(k_prep_codebook<SCOUP_BF16>, dim3(grid), dim3(256), 0, s, C, m, d, kpad, npad,
                       transposed, (uint8_t*)out, (const float*)nullptr);
  } else {
    hipLaunchKernelGGL(k_prep_codebook<SCOUP_F32>, dim3(grid), dim3(256), 0, s, C, m, d, kpad, npad,
                       transposed, (uint8_t*)out, (const float*)nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs& a, hipStream_t s, int stage) {
  const size_t lds = decode_lds_bytes(a.m, a.in_dtype);
  const long long tiles = (a.P + kDecBM - 1) / kDecBM;
  if (tiles == 0) return hipSuccess;
  const int grid = (int)std::min<long long>(tiles, kDecGrid);   // workgroups walk the tiles
  StageTimer::begin(stage, s);
  hipError_t e;
  if (decode_uses_bs(a)) {
    const int nw = decode_npad(a.d) / 32;
    const long long bt = (a.P + kBsRows - 1) / kBsRows;
    const int g = (int)std::min<long long>(bt, 256);           // one workgroup per CU
    const size_t bl = decode_bs_lds_bytes(a);
    const int ldo = a.ldo > 0 ? a.ldo : a.d;
    if (a.in_dtype == SCOUP_BF16) {
      if (a.out_dtype == SCOUP_F32) launch_bs<SCOUP_BF16, float>(a, g, nw, bl, ldo, s);
      else launch_bs<SCOUP_BF16, uint16_t>(a, g, nw, bl, ldo, s);
    } else {
      if (a.out_dtype == SCOUP_F32) launch_bs<SCOUP_FP8_E4M3, float>(a, g, nw, bl, ldo, s);
      else launch_bs<SCOUP_FP8_E4M3, uint16_t>(a, g, nw, bl, ldo, s);
    }
    StageTimer::end(stage, s);
    return hipGetLastError();
  }
  if (a.in_dtype == SCOUP_F32)
    e = a.out_dtype == SCOUP_F32 ? dispatch_nct<SCOUP_F32, float>(a, s, lds, grid)
                                 : dispatch_nct<SCOUP_F32, uint16_t>(a, s, lds, grid);
  else if (a.in_dtype == SCOUP_BF16)
    e = a.out_dtype == SCOUP_F32 ? dispatch_nct<SCOUP_BF16, float>(a, s, lds, grid)
                                 : dispatch_nct<SCOUP_BF16, uint16_t>(a, s, lds, grid);
  else
    e = a.out_dtype == SCOUP_F32 ? dispatch_nct<SCOUP_FP8_E4M3, float>(a, s, lds, grid)
                                 : dispatch_nct<SCOUP_FP8_E4M3, uint16_t>(a, s, lds, grid);
  StageTimer::end(stage, s);
  return e;
}

}  // namespace scoup
