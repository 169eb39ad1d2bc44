// Sparse coefficient render (Eq. 7) and the fused render + decode (Eq. 7
// then Eq. 8) for one camera:
//   W_hat_v(p) = sum_{i in N_{v,p}} w_hat_i e_i(v,p)       (K (atom, value) pairs per Gaussian)
//   F_v(p)     = W_hat_v(p) C                               (codebook C, M x D)
// with the front-to-back weights e of Eq. 2 (the uplift's compositing).
//
// One workgroup (4 waves) per 8x8 pixel block, its depth-ordered list from
// the binning.  The block's coefficient rows W[64][M] (float32, stride M+1)
// stay in LDS for the whole block:
//   * wave 0 composites the block's 64 pixels (one lane each) over batches of
//     kRB Gaussians and writes e into an LDS matrix E[Gaussian][pixel], with
//     the batch's code slots; double buffered, so wave 0 composites batch b+1
//     while
//   * waves 1..3 add e * value into W for batch b: wave w takes the code slots
//     whose atom is (w - 1) mod 3, so every row entry has one writer adding in
//     list order (no cross-wave atomics, bit-reproducible maps);
//   * then either the rows are written out (the coefficient map, 16-byte
//     stores, float32 / bfloat16 / FP8 E4M3) and / or the four waves decode the
//     block on MFMA, F^T = C^T W^T (wave w: D/4 feature columns), and the
//     features leave through LDS as whole 16-byte row pieces.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kRB = 16;                 // Gaussians per compositing batch
constexpr int kRKMax = 16;              // Top-K slots per Gaussian
constexpr int kRThreads = 256;          // four waves
constexpr int kRCtrl = 64;              // control words at the end of the LDS block
constexpr int kNoDecode = -1;

// LDS layout (bytes): W rows | E[2][kRB][64] | code atoms [2][kRB*kRKMax] |
// code values [2][kRB*kRKMax] | control
__host__ __device__ constexpr size_t render_rows_bytes(int m) { return (size_t)4 * 64 * (m + 1); }
__host__ __device__ constexpr size_t render_lds_total(int m) {
  return render_rows_bytes(m) + 4 * 2 * kRB * 64 + 2 * 4 * 2 * kRB * kRKMax + kRCtrl;
}

template <int T> struct RFrag;
template <> struct RFrag<SCOUP_F32> {
  static constexpr int KS = 2;
  typedef float type;
  static __device__ __forceinline__ f16v mfma(float a, float b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <> struct RFrag<SCOUP_BF16> {
  static constexpr int KS = 16;
  typedef bf16x8 type;
  static __device__ __forceinline__ f16v mfma(bf16x8 a, bf16x8 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct RFrag<SCOUP_FP8_E4M3> {
  static constexpr int KS = 64;
  typedef i32x8 type;
  static __device__ __forceinline__ f16v mfma(i32x8 a, i32x8 b, f16v c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
};

// four outputs into LDS (float32: 16 bytes, bfloat16: 8 bytes)
__device__ __forceinline__ void lds_store4(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ void lds_store4(uint16_t* p, float a, float b, float c, float d) {
  const unsigned int lo = (unsigned int)f32_to_bf16_rne(a) | ((unsigned int)f32_to_bf16_rne(b) << 16);
  const unsigned int hi = (unsigned int)f32_to_bf16_rne(c) | ((unsigned int)f32_to_bf16_rne(d) << 16);
  *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi);
}

// two workgroups per CU (the LDS of two M = 256 blocks) need at most 256
// registers per lane; 1024 feature columns (NCT = 8) need more and run one
template <int IN_T, int NCT, int WPE = (NCT <= 4 ? 2 : 1)>
__global__ __launch_bounds__(kRThreads) __attribute__((amdgpu_waves_per_eu(WPE))) void k_render_block(
    const RenderBlockArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const BinArgs& bn = a.bin;
  Status* st = bn.status;
  if (st->view_overflow) return;
  const int M = a.m_atoms, K = a.k, stride = M + 1;
  float* W = reinterpret_cast<float*>(lds);
  float* E = reinterpret_cast<float*>(lds + render_rows_bytes(M));           // [2][kRB][64]
  int* CI = reinterpret_cast<int*>(E + 2 * kRB * 64);                        // [2][kRB * kRKMax]
  float* CV = reinterpret_cast<float*>(CI + 2 * kRB * kRKMax);               // [2][kRB * kRKMax]
  int* ctrl = reinterpret_cast<int*>(CV + 2 * kRB * kRKMax);  // live[2], n_batches (ordered by the barriers)

  const int tile = (int)bn.tile_order[blockIdx.x];                          // longest lists first
  const int tx = tile % bn.tiles_x, ty = tile / bn.tiles_x;
  const int Wd = bn.cam.width, Hd = bn.cam.height;
  const unsigned int start = bn.tile_start[tile];
  const int L = (int)(bn.tile_start[tile + 1] - start);
  const unsigned long long* keys = bn.keys[bn.sorted];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tile_x0 = tx * 8, tile_y0 = ty * 8;

  for (int j = tid; j < 64 * stride; j += kRThreads) W[j] = 0.0f;
  const int nb_total = (L + kRB - 1) / kRB;
  if (tid == 0) ctrl[2] = nb_total;
  __syncthreads();

  // ---- phase A: composite (wave 0) and accumulate (waves 1..3) -------------
  const int lx = lane & 7, ly = lane >> 3;
  const bool inside = tile_x0 + lx < Wd && tile_y0 + ly < Hd;
  float T = inside ? 1.0f : -1.0f;               // wave 0: transmittance, negated once finished
  unsigned int count = 0u;
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  const int nslots = kRB * K;
  // wave 0 prefetch, three batches deep: the ids of batch b+3 are loaded while
  // batch b composites, the splats and code slots of batch b+2 (lanes < kRB
  // hold a batch's ids and splats; lane t holds code slot t mod K of Gaussian t / K)
  auto key_at = [&](int i) { return (unsigned int)keys[start + min(i, max(L - 1, 0))]; };
  auto load_data = [&](unsigned int key, GSplat& sp, int (&ci)[4], float (&cv)[4]) {
    if (lane < kRB) sp = bn.splats[key];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = min(lane + 64 * r, nslots - 1);
      const int g = t / K, s = t - g * K;
      const unsigned int id = (unsigned int)__shfl((int)key, g, 64);
      ci[r] = a.topk_idx[(long long)id * K + s];
      cv[r] = a.topk_val[(long long)id * K + s];
    }
  };
  unsigned int key2 = 0u;
  GSplat sp0, sp1;
  int ci0[4], ci1[4];
  float cv0[4], cv1[4];
  if (wave == 0 && L > 0) {
    const unsigned int k0 = key_at(lane & (kRB - 1)), k1 = key_at(kRB + (lane & (kRB - 1)));
    key2 = key_at(2 * kRB + (lane & (kRB - 1)));
    load_data(k0, sp0, ci0, cv0);
    load_data(k1, sp1, ci1, cv1);
  }

  int nb_run = nb_total;
  for (int it = 0; it <= nb_run; ++it) {
    const int buf = it & 1;
    if (wave == 0) {
      if (it < nb_run) {
        const int b0 = it * kRB;
        const int nb = min(kRB, L - b0);
        BlockSplat mine;
        if (lane < kRB) {
          mine.load(sp0, tile_x0, tile_y0);
          if (lane >= nb) mine.qmax = -1.0f;           // past the list: never taken (q >= 0)
        }
        int* ci = CI + buf * kRB * kRKMax;
        float* cv = CV + buf * kRB * kRKMax;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int t = lane + 64 * r;
          if (t < nb * K) { ci[t] = ci0[r]; cv[t] = cv0[r]; }
        }
        // loads of batch it+2 (splats, codes) and it+3 (ids) in flight during this batch
        GSplat sp2;
        int ci2[4];
        float cv2[4];
        const bool more = b0 + 2 * kRB < L;
        unsigned int key3 = key2;
        if (more) {
          load_data(key2, sp2, ci2, cv2);
          key3 = key_at(b0 + 3 * kRB + (lane & (kRB - 1)));
        }
        float* e_out = E + buf * kRB * 64;
        unsigned int kept = 0u;                      // bit g: this lane's pixel took Gaussian g
        // unrolled: alpha of later Gaussians does not depend on T, so only the
        // short T chain is sequential
#pragma unroll
        for (int g = 0; g < kRB; ++g) {
          const BlockSplat s = mine.bcast(g);
          const float dx = (pcx - s.hx) - s.fx, dy = (pcy - s.hy) - s.fy;
          const float u = fmaf(s.l00, dx, s.l10 * dy), v = s.l11 * dy;
          const float q = fmaf(u, u, v * v);
          // branchless front-to-back step (the uplift's); a finished pixel keeps -T
          const float alpha = fminf(kAlphaMax, s.opacity * __builtin_amdgcn_exp2f(-q));
          const float testT = T * (1.0f - alpha);
          const bool take = T > 0.0f && q <= s.qmax;
          const bool keep = take && testT >= kTMin;
          const float e = keep ? alpha * T : 0.0f;
          T = take ? (keep ? testT : -T) : T;
          kept |= keep ? (1u << g) : 0u;
          e_out[g * 64 + lane] = e;
        }
        count += (unsigned int)__popc(kept);
        unsigned int live = kept;                    // OR over the wave: Gaussians with a contribution
        for (int o = 32; o >= 1; o >>= 1) live |= (unsigned int)__shfl_xor((int)live, o, 64);
        sp0 = sp1;
#pragma unroll
        for (int r = 0; r < 4; ++r) { ci0[r] = ci1[r]; cv0[r] = cv1[r]; }
        if (more) {
          sp1 = sp2;
#pragma unroll
          for (int r = 0; r < 4; ++r) { ci1[r] = ci2[r]; cv1[r] = cv2[r]; }
          key2 = key3;
        }
        const bool finished = __ballot(T > 0.0f) == 0ull;      // every pixel of the block
        if (lane == 0) {
          ctrl[buf] = (int)live;
          if (finished) ctrl[2] = it + 1;
        }
      }
    } else if (it > 0) {
      // accumulate batch it-1: this wave's code slots (atom % 3 == wave - 1), in
      // list order.  The batch's e (this lane's pixel) and code slots (lane s:
      // slot s of every Gaussian) are read into registers first, so the adds
      // below wait on no memory.
      const int pb = buf ^ 1;
      const unsigned int live = (unsigned int)ctrl[pb];
      const int nbp = min(kRB, L - (it - 1) * kRB);
      const int* ci = CI + pb * kRB * kRKMax;
      const float* cv = CV + pb * kRB * kRKMax;
      const float* e_in = E + pb * kRB * 64;
      float* myrow = W + lane * stride;
      const int cls = wave - 1;
      const int sl = lane < K ? lane : 0;
      float ev[kRB], vr[kRB];
      int jr[kRB];
#pragma unroll
      for (int g = 0; g < kRB; ++g) {
        ev[g] = e_in[g * 64 + lane];
        jr[g] = ci[g * K + sl];
        vr[g] = cv[g * K + sl];
      }
#pragma unroll
      for (int g = 0; g < kRB; ++g) {
        if (g >= nbp || !((live >> g) & 1u)) continue;     // uniform
        const int j = jr[g];
        if (cls == 0 && __ballot(lane < K && j >= M)) atomicOr(&st->data_error, 4u);
        unsigned long long todo = __ballot(lane < K && j >= 0 && j < M && (j % 3) == cls);
        const float eg = ev[g];
        const bool add = eg != 0.0f;                 // lanes whose pixel took g
        while (todo) {
          const int sidx = __ffsll((long long)todo) - 1;
          todo &= todo - 1ull;
          const int jj = __builtin_amdgcn_readlane(j, sidx);
          const float vv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vr[g]), sidx));
          if (add) myrow[jj] += eg * vv;         // one writer per row entry: no atomic needed
        }
      }
    }
    __syncthreads();
    nb_run = ctrl[2];
  }
  if (wave == 0) {
    if (inside && a.t_final) a.t_final[(long long)(tile_y0 + ly) * Wd + tile_x0 + lx] = fabsf(T);
    unsigned long long total = count;
    for (int o = 32; o >= 1; o >>= 1) total += __shfl_xor(total, o, 64);
    if (lane == 0 && total) atomicAdd(&st->contrib, total);
  }

  // ---- phase B1: the coefficient map, 16-byte pieces of whole pixel rows ---
  if (a.map) {
    const int es = a.map_dtype == SCOUP_F32 ? 4 : a.map_dtype == SCOUP_BF16 ? 2 : 1;
    const int per = 16 / es;                       // values per 16-byte piece
    const long long row_bytes = (long long)M * es;
    const bool vec = (row_bytes & 15) == 0 && (reinterpret_cast<uintptr_t>(a.map) & 15) == 0;
    uint8_t* mbase = reinterpret_cast<uint8_t*>(a.map);
    if (vec) {
      const int pieces = M / per;
      for (int c = tid; c < 64 * pieces; c += kRThreads) {
        const int p = c / pieces, q = c - p * pieces;
        const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
        if (ox >= Wd || oy >= Hd) continue;
        const float* src = W + p * stride + q * per;
        i32x4 v;
        if (a.map_dtype == SCOUP_F32) {
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = __float_as_int(src[u] * a.map_scale);
        } else if (a.map_dtype == SCOUP_BF16) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            v[u] = (int)((unsigned int)f32_to_bf16_rne(src[2 * u] * a.map_scale) |
                         ((unsigned int)f32_to_bf16_rne(src[2 * u + 1] * a.map_scale) << 16));
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            v[u] = (int)((unsigned int)f32_to_e4m3(src[4 * u] * a.map_scale) |
                         ((unsigned int)f32_to_e4m3(src[4 * u + 1] * a.map_scale) << 8) |
                         ((unsigned int)f32_to_e4m3(src[4 * u + 2] * a.map_scale) << 16) |
                         ((unsigned int)f32_to_e4m3(src[4 * u + 3] * a.map_scale) << 24));
        }
        *reinterpret_cast<i32x4*>(mbase + ((long long)oy * Wd + ox) * row_bytes + q * 16) = v;
      }
    } else {
      for (int c = tid; c < 64 * M; c += kRThreads) {
        const int p = c / M, j = c - p * M;
        const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
        if (ox >= Wd || oy >= Hd) continue;
        const long long o = ((long long)oy * Wd + ox) * M + j;
        const float v = W[p * stride + j] * a.map_scale;
        if (a.map_dtype == SCOUP_F32) reinterpret_cast<float*>(mbase)[o] = v;
        else if (a.map_dtype == SCOUP_BF16) reinterpret_cast<uint16_t*>(mbase)[o] = f32_to_bf16_rne(v);
        else mbase[o] = f32_to_e4m3(v);
      }
    }
  }

  // ---- phase B2: decode F^T = C^T W^T on MFMA ------------------------------
  if constexpr (IN_T != kNoDecode) {
    using FR = RFrag<IN_T>;
    using FT = typename FR::type;
    const int nks = a.kpad / FR::KS;
    const int ct0 = wave * NCT;                    // this wave's 32-column tiles (D/4 columns)
    const FT* Bf = reinterpret_cast<const FT*>(a.codebook_prep);
    float mul = a.out_mul;
    if (a.cb_scale) mul /= *a.cb_scale;
    f16v acc[2][NCT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < NCT; ++c) acc[h][c] = (f16v){};
    // FP8 operands are converted once into LDS (the batch buffers are free now), 128 atoms at a time
    uint8_t* q8 = reinterpret_cast<uint8_t*>(E);
    constexpr int kQ8Row = 128 + 16;
    const int k_chunk = IN_T == SCOUP_FP8_E4M3 ? 128 : a.kpad;
    for (int kb = 0; kb < a.kpad; kb += k_chunk) {
      if constexpr (IN_T == SCOUP_FP8_E4M3) {
        __syncthreads();
        for (int c = tid; c < 64 * 32; c += kRThreads) {      // 64 rows x 32 four-byte words
          const int p = c >> 5, w4 = c & 31;
          unsigned int word = 0u;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = kb + 4 * w4 + u;
            const float x = j < M ? W[p * stride + j] * a.q_scale : 0.0f;
            word |= (unsigned int)f32_to_e4m3(x) << (8 * u);
          }
          *reinterpret_cast<unsigned int*>(q8 + p * kQ8Row + 4 * w4) = word;
        }
        __syncthreads();
      }
      const int ks0 = kb / FR::KS, ks1 = min(nks, (kb + k_chunk) / FR::KS);
      FT bcur[NCT];
#pragma unroll
      for (int c = 0; c < NCT; ++c) bcur[c] = Bf[((long long)(ct0 + c) * nks + ks0) * 64 + lane];
      // codebook fragments one k-step ahead (not for FP8: its wider fragments
      // would take the registers two workgroups per CU leave)
      constexpr bool kAhead = IN_T != SCOUP_FP8_E4M3;
      for (int ks = ks0; ks < ks1; ++ks) {
        FT bnext[NCT];
        if (kAhead && ks + 1 < ks1) {
#pragma unroll
          for (int c = 0; c < NCT; ++c) bnext[c] = Bf[((long long)(ct0 + c) * nks + ks + 1) * 64 + lane];
        }
        FT af[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int p = h * 32 + (lane & 31);
          if constexpr (IN_T == SCOUP_F32) {
            const int j = ks * 2 + (lane >> 5);
            af[h] = j < M ? W[p * stride + j] : 0.0f;
          } else if constexpr (IN_T == SCOUP_BF16) {
            const int j0 = ks * 16 + (lane >> 5) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const float x = j0 + u < M ? W[p * stride + j0 + u] : 0.0f;
              af[h][u] = __builtin_bit_cast(__bf16, f32_to_bf16_rne(x));
            }
          } else {
            const int jb = ks * 64 - kb + (lane >> 5) * 32;
            af[h] = *reinterpret_cast<const i32x8*>(q8 + p * kQ8Row + jb);
          }
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          acc[0][c] = FR::mfma(bcur[c], af[0], acc[0][c]);
          acc[1][c] = FR::mfma(bcur[c], af[1], acc[1][c]);
        }
        if (ks + 1 < ks1) {
#pragma unroll
          for (int c = 0; c < NCT; ++c)
            bcur[c] = kAhead ? bnext[c] : Bf[((long long)(ct0 + c) * nks + ks + 1) * 64 + lane];
        }
      }
    }
    __syncthreads();                               // every wave has read W: its LDS now stages features
    // element r of lane l in a 32x32 tile of F^T: feature (ct0+c)*32 + 8(r/4) + 4(l/32) + r%4,
    // pixel h*32 + l%32; `rows` pixels at a time, each row (npad x out bytes + 16) long
    const int OES = a.out_dtype == SCOUP_F32 ? 4 : 2;
    const int D = a.d;
    const int srow = a.npad * OES + 16;
    constexpr int rows = 32;
    const bool vec = ((long long)D * OES) % 16 == 0 && (reinterpret_cast<uintptr_t>(a.features) & 15) == 0;
    uint8_t* fbase = reinterpret_cast<uint8_t*>(a.features);
    for (int p0 = 0; p0 < 64; p0 += rows) {
      const int h = p0 >> 5;
      const int pl = (lane & 31) + 32 * h;         // this lane's pixel in the block
      if (pl >= p0 && pl < p0 + rows) {
        uint8_t* row = lds + (pl - p0) * srow;
#pragma unroll
        for (int c = 0; c < NCT; ++c)
#pragma unroll
          for (int rg = 0; rg < 4; ++rg) {
            const int d0 = (ct0 + c) * 32 + 8 * rg + 4 * (lane >> 5);
            const f16v v = h == 0 ? acc[0][c] : acc[1][c];
            if (OES == 4)
              lds_store4(reinterpret_cast<float*>(row) + d0, v[4 * rg] * mul, v[4 * rg + 1] * mul,
                         v[4 * rg + 2] * mul, v[4 * rg + 3] * mul);
            else
              lds_store4(reinterpret_cast<uint16_t*>(row) + d0, v[4 * rg] * mul, v[4 * rg + 1] * mul,
                         v[4 * rg + 2] * mul, v[4 * rg + 3] * mul);
          }
      }
      __syncthreads();
      if (vec) {
        const int pieces = D * OES / 16;
        for (int c = tid; c < rows * pieces; c += kRThreads) {
          const int r = c / pieces, q = c - r * pieces;
          const int p = p0 + r;
          const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
          if (ox >= Wd || oy >= Hd) continue;
          *reinterpret_cast<i32x4*>(fbase + ((long long)oy * Wd + ox) * D * OES + q * 16) =
              *reinterpret_cast<const i32x4*>(lds + r * srow + q * 16);
        }
      } else {
        for (int c = tid; c < rows * D; c += kRThreads) {
          const int r = c / D, d = c - r * D;
          const int p = p0 + r;
          const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
          if (ox >= Wd || oy >= Hd) continue;
          const long long o = ((long long)oy * Wd + ox) * D + d;
          if (OES == 4) reinterpret_cast<float*>(fbase)[o] = reinterpret_cast<const float*>(lds + r * srow)[d];
          else reinterpret_cast<uint16_t*>(fbase)[o] = reinterpret_cast<const uint16_t*>(lds + r * srow)[d];
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// The fused render + decode at BF16 / FP8 precision accumulates the block's
// coefficient rows on MFMA instead of LDS adds.  Per batch of kRB Gaussians
//   W^T[atoms][pixels] += What^T[atoms][Gaussians] E[Gaussians][pixels]
// is one v_mfma_f32_32x32x16_bf16 per 32x32 tile (the batch is the k-step),
// with e and the Top-K values rounded to bfloat16 -- the decode's input
// precision -- and float32 accumulation.  Wave w holds the 32-atom tiles
// w, w+4, ... of W^T for the block's 64 pixels in registers; wave 0 also
// composites (E^T written as bfloat16, double buffered); each wave scatters
// the batch's code slots of its own atoms into a small dense What^T slice in
// LDS, multiplies, and clears the slice again.  No LDS is held for float32
// rows, so more blocks share a CU.  After the list, W is written to LDS in the
// decode's precision and the block is decoded as in k_render_block.
// ---------------------------------------------------------------------------
constexpr int kMxRow = 24;                       // bf16 per E^T / What^T row: 16 + 8 (conflict-free 16-byte reads)

__host__ __device__ constexpr size_t mx_region_a(int tpw) {
  return (size_t)2 * 64 * kMxRow * 2 + (size_t)4 * tpw * 32 * kMxRow * 2 + 2 * 4 * 2 * kRB * kRKMax;
}
// bytes per pixel row of W in the decode's precision: the decode's k range (kpad)
// and every atom of the 32-atom tiles, plus 16 bytes against bank conflicts
__host__ __device__ constexpr int mx_wrow(int kpad, int m, int in_t) {
  return in_t == SCOUP_BF16 ? ((kpad > (m + 31) / 32 * 32 ? kpad : (m + 31) / 32 * 32) + 8) * 2
                            : (kpad > (m + 31) / 32 * 32 ? kpad : (m + 31) / 32 * 32) + 16;
}
__host__ __device__ constexpr size_t mx_region_b(int kpad, int m, int npad, int in_t, int out_t) {
  // W rows, then the staging of one pass: 32 rows of 4 NCH x 32 features
  return ((64 * (size_t)mx_wrow(kpad, m, in_t) + 15) & ~(size_t)15) +
         (size_t)32 * ((size_t)4 * (npad / 128 <= 2 ? npad / 128 : 2) * 32 * (out_t == SCOUP_F32 ? 4 : 2) + 16);
}
size_t render_mx_lds_bytes(int m, int kpad, int npad, int in_t, int out_t) {
  const int tpw = ((m + 31) / 32 + 3) / 4;
  return std::max(mx_region_a(tpw <= 1 ? 1 : tpw <= 2 ? 2 : 4), mx_region_b(kpad, m, npad, in_t, out_t)) + kRCtrl;
}

// three workgroups per CU (at most 168 registers) for BF16 up to 256 atoms;
// two otherwise (FP8's conversion of the rows needs more registers)
template <int IN_T, int NCT, int TPW, int WPE = (TPW <= 2 && IN_T == SCOUP_BF16 ? 3 : 2)>
__global__ __launch_bounds__(kRThreads) __attribute__((amdgpu_waves_per_eu(WPE))) void k_render_mx(
    const RenderBlockArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const BinArgs& bn = a.bin;
  Status* st = bn.status;
  if (st->view_overflow) return;
  const int M = a.m_atoms, K = a.k;
  const size_t ra = mx_region_a(TPW);
  const int wrow = mx_wrow(a.kpad, M, IN_T);
  const size_t rb = mx_region_b(a.kpad, M, a.npad, IN_T, a.out_dtype);
  uint16_t* Et = reinterpret_cast<uint16_t*>(lds);                          // [2][64][kMxRow]
  uint16_t* Wh = Et + 2 * 64 * kMxRow;                                       // [4][TPW*32][kMxRow]
  int* CI = reinterpret_cast<int*>(Wh + 4 * TPW * 32 * kMxRow);             // [2][kRB * kRKMax]
  float* CV = reinterpret_cast<float*>(CI + 2 * kRB * kRKMax);
  int* ctrl = reinterpret_cast<int*>(lds + std::max(ra, rb));

  const int tile = (int)bn.tile_order[blockIdx.x];
  const int tx = tile % bn.tiles_x, ty = tile / bn.tiles_x;
  const int Wd = bn.cam.width, Hd = bn.cam.height;
  const unsigned int start = bn.tile_start[tile];
  const int L = (int)(bn.tile_start[tile + 1] - start);
  const unsigned long long* keys = bn.keys[bn.sorted];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tile_x0 = tx * 8, tile_y0 = ty * 8;
  const int ntiles = (M + 31) / 32;                 // 32-atom tiles; wave w owns w, w+4, ...
  uint16_t* myWh = Wh + wave * TPW * 32 * kMxRow;
  for (int j = lane; j < TPW * 32 * kMxRow; j += 64) myWh[j] = 0;
  const int nb_total = (L + kRB - 1) / kRB;
  if (tid == 0) ctrl[2] = nb_total;
  __syncthreads();

  f16v acc[TPW][2];
#pragma unroll
  for (int t = 0; t < TPW; ++t) { acc[t][0] = (f16v){}; acc[t][1] = (f16v){}; }

  const int lx = lane & 7, ly = lane >> 3;
  const bool inside = tile_x0 + lx < Wd && tile_y0 + ly < Hd;
  float T = inside ? 1.0f : -1.0f;
  unsigned int count = 0u;
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  const int nslots = kRB * K;
  // wave 0 prefetch: ids two batches ahead, splats and code slots one batch ahead
  auto key_at = [&](int i) { return (unsigned int)keys[start + min(i, max(L - 1, 0))]; };
  auto load_data = [&](unsigned int key, GSplat& sp, int (&ci)[4], float (&cv)[4]) {
    if (lane < kRB) sp = bn.splats[key];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = min(lane + 64 * r, nslots - 1);
      const int g = t / K, s = t - g * K;
      const unsigned int id = (unsigned int)__shfl((int)key, g, 64);
      ci[r] = a.topk_idx[(long long)id * K + s];
      cv[r] = a.topk_val[(long long)id * K + s];
    }
  };
  unsigned int key1 = 0u;
  GSplat sp0;
  int ci0[4];
  float cv0[4];
  if (wave == 0 && L > 0) {
    load_data(key_at(lane & (kRB - 1)), sp0, ci0, cv0);
    key1 = key_at(kRB + (lane & (kRB - 1)));
  }

  int nb_run = nb_total;
  for (int it = 0; it <= nb_run; ++it) {
    const int buf = it & 1;
    if (wave == 0 && it < nb_run) {
      const int b0 = it * kRB;
      const int nb = min(kRB, L - b0);
      BlockSplat mine;
      if (lane < kRB) {
        mine.load(sp0, tile_x0, tile_y0);
        if (lane >= nb) mine.qmax = -1.0f;
      }
      int* ci = CI + buf * kRB * kRKMax;
      float* cv = CV + buf * kRB * kRKMax;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = lane + 64 * r;
        if (t < nb * K) { ci[t] = ci0[r]; cv[t] = cv0[r]; }
      }
      GSplat sp1;
      int ci1[4];
      float cv1[4];
      const bool more = b0 + kRB < L;
      unsigned int key2 = key1;
      if (more) {
        load_data(key1, sp1, ci1, cv1);
        key2 = key_at(b0 + 2 * kRB + (lane & (kRB - 1)));
      }
      unsigned int kept = 0u, ep[kRB / 2];
#pragma unroll
      for (int g = 0; g < kRB; ++g) {
        const BlockSplat s = mine.bcast(g);
        const float dx = (pcx - s.hx) - s.fx, dy = (pcy - s.hy) - s.fy;
        const float u = fmaf(s.l00, dx, s.l10 * dy), v = s.l11 * dy;
        const float q = fmaf(u, u, v * v);
        const float alpha = fminf(kAlphaMax, s.opacity * __builtin_amdgcn_exp2f(-q));
        const float testT = T * (1.0f - alpha);
        const bool take = T > 0.0f && q <= s.qmax;
        const bool keep = take && testT >= kTMin;
        const float e = keep ? alpha * T : 0.0f;
        T = take ? (keep ? testT : -T) : T;
        kept |= keep ? (1u << g) : 0u;
        const unsigned int eb = f32_to_bf16_rne(e);
        if (g & 1) ep[g >> 1] |= eb << 16; else ep[g >> 1] = eb;
      }
      // this pixel's row of E^T: 16 bfloat16 = two 16-byte stores
      uint4* erow = reinterpret_cast<uint4*>(Et + (buf * 64 + lane) * kMxRow);
      erow[0] = make_uint4(ep[0], ep[1], ep[2], ep[3]);
      erow[1] = make_uint4(ep[4], ep[5], ep[6], ep[7]);
      count += (unsigned int)__popc(kept);
      unsigned int live = kept;
      for (int o = 32; o >= 1; o >>= 1) live |= (unsigned int)__shfl_xor((int)live, o, 64);
      const bool finished = __ballot(T > 0.0f) == 0ull;
      if (lane == 0) {
        ctrl[buf] = (int)live;
        if (finished) ctrl[2] = it + 1;
      }
      if (more) {
        sp0 = sp1;
#pragma unroll
        for (int r = 0; r < 4; ++r) { ci0[r] = ci1[r]; cv0[r] = cv1[r]; }
        key1 = key2;
      }
    }
    if (it > 0) {
      // batch it-1: scatter this wave's code slots into its What^T slice, one
      // MFMA per (atom tile, pixel half), clear the slice again
      const int pb = buf ^ 1;
      const unsigned int live = (unsigned int)ctrl[pb];
      const int nbk = min(kRB, L - (it - 1) * kRB) * K;
      const int* ci = CI + pb * kRB * kRKMax;
      const float* cv = CV + pb * kRB * kRKMax;
      int slot[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = lane + 64 * r;
        slot[r] = -1;
        if (t < nbk) {
          const int g = t / K;
          const int j = ci[t];
          if (j >= M && wave == 0) atomicOr(&st->data_error, 4u);
          if (((live >> g) & 1u) && j >= 0 && j < M && ((j >> 5) & 3) == wave) {
            slot[r] = (((j >> 5) >> 2) * 32 + (j & 31)) * kMxRow + g;
            myWh[slot[r]] = f32_to_bf16_rne(cv[t]);
          }
        }
      }
      const uint16_t* ebase = Et + pb * 64 * kMxRow;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (wave + 4 * t >= ntiles) break;
        const bf16x8 A = *reinterpret_cast<const bf16x8*>(myWh + (t * 32 + (lane & 31)) * kMxRow + 8 * (lane >> 5));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bf16x8 B = *reinterpret_cast<const bf16x8*>(ebase + (h * 32 + (lane & 31)) * kMxRow + 8 * (lane >> 5));
          acc[t][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[t][h], 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (slot[r] >= 0) myWh[slot[r]] = 0;
    }
    __syncthreads();
    nb_run = ctrl[2];
  }
  if (wave == 0) {
    if (inside && a.t_final) a.t_final[(long long)(tile_y0 + ly) * Wd + tile_x0 + lx] = fabsf(T);
    unsigned long long total = count;
    for (int o = 32; o >= 1; o >>= 1) total += __shfl_xor(total, o, 64);
    if (lane == 0 && total) atomicAdd(&st->contrib, total);
  }

  // W in the decode's precision: pixel rows of kpad atoms (zero past the tiles)
  uint8_t* Wq = lds;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tl = wave + 4 * t;
    if (tl >= ntiles) break;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = h * 32 + (lane & 31);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j0 = tl * 32 + 8 * q + 4 * (lane >> 5);
        const f16v& v = acc[t][h];
        if constexpr (IN_T == SCOUP_BF16) {
          const unsigned int lo = (unsigned int)f32_to_bf16_rne(v[4 * q]) | ((unsigned int)f32_to_bf16_rne(v[4 * q + 1]) << 16);
          const unsigned int hi = (unsigned int)f32_to_bf16_rne(v[4 * q + 2]) | ((unsigned int)f32_to_bf16_rne(v[4 * q + 3]) << 16);
          *reinterpret_cast<uint2*>(Wq + p * wrow + 2 * j0) = make_uint2(lo, hi);
        } else {
          const unsigned int w4 = (unsigned int)f32_to_e4m3(v[4 * q] * a.q_scale) |
                                  ((unsigned int)f32_to_e4m3(v[4 * q + 1] * a.q_scale) << 8) |
                                  ((unsigned int)f32_to_e4m3(v[4 * q + 2] * a.q_scale) << 16) |
                                  ((unsigned int)f32_to_e4m3(v[4 * q + 3] * a.q_scale) << 24);
          *reinterpret_cast<unsigned int*>(Wq + p * wrow + j0) = w4;
        }
      }
    }
  }
  const int es = IN_T == SCOUP_BF16 ? 2 : 1;
  for (int c = tid; c < 64 * (a.kpad - ntiles * 32); c += kRThreads) {      // k padding past the tiles
    const int p = c / (a.kpad - ntiles * 32), j = ntiles * 32 + c % (a.kpad - ntiles * 32);
    for (int b = 0; b < es; ++b) Wq[p * wrow + j * es + b] = 0;
  }
  __syncthreads();

  using FR = RFrag<IN_T>;
  using FT = typename FR::type;
  const int nks = a.kpad / FR::KS;
  const FT* Bf = reinterpret_cast<const FT*>(a.codebook_prep);
  float mul = a.out_mul;
  if (a.cb_scale) mul /= *a.cb_scale;
  const int OES = a.out_dtype == SCOUP_F32 ? 4 : 2;
  const int D = a.d;
  // passes of NCH column tiles per wave (fewer live accumulators): pass ps,
  // wave w owns tiles (4 ps + w) NCH .. +NCH-1, so a pass covers 4 NCH x 32
  // consecutive features; they are staged 32 pixels at a time past W's rows
  constexpr int NCH = NCT <= 2 ? NCT : 2;
  constexpr int PCOLS = 4 * NCH * 32;
  const int srow = PCOLS * OES + 16;
  uint8_t* stage = lds + ((64 * (size_t)wrow + 15) & ~(size_t)15);
  uint8_t* fbase = reinterpret_cast<uint8_t*>(a.features);
  for (int ps = 0; ps < NCT / NCH; ++ps) {
    const int ct0 = (4 * ps + wave) * NCH;
    f16v fo[2][NCH];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < NCH; ++c) fo[h][c] = (f16v){};
    FT bcur[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) bcur[c] = Bf[((long long)(ct0 + c) * nks) * 64 + lane];
    for (int ks = 0; ks < nks; ++ks) {
      FT bnext[NCH];
      if (ks + 1 < nks) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) bnext[c] = Bf[((long long)(ct0 + c) * nks + ks + 1) * 64 + lane];
      }
      FT af[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = h * 32 + (lane & 31);
        af[h] = *reinterpret_cast<const FT*>(Wq + p * wrow + (ks * FR::KS + (lane >> 5) * (FR::KS / 2)) * es);
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        fo[0][c] = FR::mfma(bcur[c], af[0], fo[0][c]);
        fo[1][c] = FR::mfma(bcur[c], af[1], fo[1][c]);
      }
      if (ks + 1 < nks) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) bcur[c] = bnext[c];
      }
    }
    const int col0 = ps * PCOLS;                 // first feature column of the pass
    const int ncol = min(PCOLS, D - col0);       // valid columns of the pass
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint8_t* row = stage + (lane & 31) * srow;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
          const int d0 = (wave * NCH + c) * 32 + 8 * rg + 4 * (lane >> 5);   // column within the pass
          const f16v& v = fo[h][c];
          if (OES == 4)
            lds_store4(reinterpret_cast<float*>(row) + d0, v[4 * rg] * mul, v[4 * rg + 1] * mul,
                       v[4 * rg + 2] * mul, v[4 * rg + 3] * mul);
          else
            lds_store4(reinterpret_cast<uint16_t*>(row) + d0, v[4 * rg] * mul, v[4 * rg + 1] * mul,
                       v[4 * rg + 2] * mul, v[4 * rg + 3] * mul);
        }
      __syncthreads();
      if (ncol > 0) {
        const bool vec = ((long long)D * OES) % 16 == 0 && (ncol * OES) % 16 == 0 &&
                         (reinterpret_cast<uintptr_t>(a.features) & 15) == 0;
        if (vec) {
          const int pieces = ncol * OES / 16;
          for (int c = tid; c < 32 * pieces; c += kRThreads) {
            const int r = c / pieces, q = c - r * pieces;
            const int p = h * 32 + r;
            const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
            if (ox >= Wd || oy >= Hd) continue;
            *reinterpret_cast<i32x4*>(fbase + (((long long)oy * Wd + ox) * D + col0) * OES + q * 16) =
                *reinterpret_cast<const i32x4*>(stage + r * srow + q * 16);
          }
        } else {
          for (int c = tid; c < 32 * ncol; c += kRThreads) {
            const int r = c / ncol, d = c - r * ncol;
            const int p = h * 32 + r;
            const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
            if (ox >= Wd || oy >= Hd) continue;
            const long long o = ((long long)oy * Wd + ox) * D + col0 + d;
            if (OES == 4) reinterpret_cast<float*>(fbase)[o] = reinterpret_cast<const float*>(stage + r * srow)[d];
            else reinterpret_cast<uint16_t*>(fbase)[o] = reinterpret_cast<const uint16_t*>(stage + r * srow)[d];
          }
        }
      }
      __syncthreads();
    }
  }
}

// feature rows of the decode are staged 32 at a time, each (npad x out bytes + 16) long;
// the LDS block covers the larger of the render's needs and that staging
size_t render_block_lds_bytes(int m, int npad, int out_dtype) {
  const size_t stage = npad > 0 ? 32 * ((size_t)npad * (out_dtype == SCOUP_F32 ? 4 : 2) + 16) + kRCtrl : 0;
  return std::max(render_lds_total(m), stage);
}

template <int IN_T, int NCT>
static void launch_rb(const RenderBlockArgs& a, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k_render_block<IN_T, NCT>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a);
}

template <int IN_T>
static hipError_t launch_rb_nct(const RenderBlockArgs& a, size_t lds, hipStream_t s) {
  switch (a.npad / 128) {
    case 1: launch_rb<IN_T, 1>(a, lds, s); break;
    case 2: launch_rb<IN_T, 2>(a, lds, s); break;
    case 4: launch_rb<IN_T, 4>(a, lds, s); break;
    case 8: launch_rb<IN_T, 8>(a, lds, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <int IN_T, int NCT>
static void launch_mx_tpw(const RenderBlockArgs& a, size_t lds, hipStream_t s) {
  const int tpw = ((a.m_atoms + 31) / 32 + 3) / 4;
  if (tpw <= 1)
    hipLaunchKernelGGL((k_render_mx<IN_T, NCT, 1>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a);
  else if (tpw <= 2)
    hipLaunchKernelGGL((k_render_mx<IN_T, NCT, 2>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a);
  else
    hipLaunchKernelGGL((k_render_mx<IN_T, NCT, 4>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a);
}

template <int IN_T>
static hipError_t launch_mx(const RenderBlockArgs& a, hipStream_t s) {
  const size_t lds = render_mx_lds_bytes(a.m_atoms, a.kpad, a.npad, IN_T, a.out_dtype);
  switch (a.npad / 128) {
    case 1: launch_mx_tpw<IN_T, 1>(a, lds, s); break;
    case 2: launch_mx_tpw<IN_T, 2>(a, lds, s); break;
    case 4: launch_mx_tpw<IN_T, 4>(a, lds, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

bool render_uses_mx(const RenderBlockArgs& a) {
  return (a.in_dtype == SCOUP_BF16 || a.in_dtype == SCOUP_FP8_E4M3) && a.npad <= 512 && !a.map;
}

hipError_t launch_render_block(RenderBlockArgs& a, hipStream_t s, int stage) {
  hipError_t e = launch_bin_view(a.bin, s);
  if (e != hipSuccess) return e;
  if (a.bin.n_tiles == 0) return hipSuccess;
  if (render_uses_mx(a)) {
    StageTimer::begin(stage, s);
    e = a.in_dtype == SCOUP_BF16 ? launch_mx<SCOUP_BF16>(a, s) : launch_mx<SCOUP_FP8_E4M3>(a, s);
    StageTimer::end(stage, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  const size_t lds = render_block_lds_bytes(a.m_atoms, a.in_dtype >= 0 ? a.npad : 0, a.out_dtype);
  StageTimer::begin(stage, s);
  switch (a.in_dtype) {
    case SCOUP_F32: e = launch_rb_nct<SCOUP_F32>(a, lds, s); break;
    case SCOUP_BF16: e = launch_rb_nct<SCOUP_BF16>(a, lds, s); break;
    case SCOUP_FP8_E4M3: e = launch_rb_nct<SCOUP_FP8_E4M3>(a, lds, s); break;
    default: launch_rb<kNoDecode, 1>(a, lds, s); break;
  }
  StageTimer::end(stage, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <int IN_T, int NCT>
static hipError_t set_rb_lds() {
  return hipFuncSetAttribute((const void*)k_render_block<IN_T, NCT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

template <int IN_T>
static hipError_t set_rb_lds_all() {
  hipError_t e;
  if ((e = set_rb_lds<IN_T, 1>()) != hipSuccess) return e;
  if ((e = set_rb_lds<IN_T, 2>()) != hipSuccess) return e;
  if ((e = set_rb_lds<IN_T, 4>()) != hipSuccess) return e;
  return set_rb_lds<IN_T, 8>();
}

template <int IN_T, int NCT, int TPW>
static hipError_t set_mx_lds() {
  return hipFuncSetAttribute((const void*)k_render_mx<IN_T, NCT, TPW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

template <int IN_T>
static hipError_t set_mx_lds_all() {
  hipError_t e;
#define SET_MX(N)                                                           \
  if ((e = set_mx_lds<IN_T, N, 1>()) != hipSuccess) return e;              \
  if ((e = set_mx_lds<IN_T, N, 2>()) != hipSuccess) return e;              \
  if ((e = set_mx_lds<IN_T, N, 4>()) != hipSuccess) return e;
  SET_MX(1) SET_MX(2) SET_MX(4)
#undef SET_MX
  return hipSuccess;
}

hipError_t render_set_lds_limits() {
  hipError_t e;
  if ((e = set_mx_lds_all<SCOUP_BF16>()) != hipSuccess) return e;
  if ((e = set_mx_lds_all<SCOUP_FP8_E4M3>()) != hipSuccess) return e;
  if ((e = set_rb_lds<kNoDecode, 1>()) != hipSuccess) return e;
  if ((e = set_rb_lds_all<SCOUP_F32>()) != hipSuccess) return e;
  if ((e = set_rb_lds_all<SCOUP_BF16>()) != hipSuccess) return e;
  return set_rb_lds_all<SCOUP_FP8_E4M3>();
}

}  // namespace scoup
