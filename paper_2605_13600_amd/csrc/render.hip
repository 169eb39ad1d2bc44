// Sparse coefficient render (Eq. 7) and the render fused with the decode
// (Eq. 7 then Eq. 8) for one camera:
//   W_hat_v(p) = sum_{i in N_{v,p}} w_hat_i e_i(v,p)       (K (atom, value) pairs per Gaussian)
//   F_v(p)     = W_hat_v(p) C                               (codebook C, M x D)
// with the front-to-back weights e of Eq. 2 (the uplift's compositing).
//
// One workgroup (4 waves) per 8x8 pixel block, its depth-ordered list from
// the binning, in batches of kRB Gaussians.  The block's coefficient rows are
// accumulated on the matrix cores: per batch
//   W^T[atoms][pixels] += What^T[atoms][Gaussians] E[Gaussians][pixels]
// Wave w holds the 32-atom tiles w, w+4, ... of W^T for the block's 64 pixels
// in its accumulators; wave 0 also composites the block (one lane per pixel,
// the batch's weights written to LDS, double buffered, so wave 0 composites
// batch b+1 while the others multiply batch b); each wave scatters the
// batch's code slots of its own atoms into a small dense What^T slice in LDS,
// multiplies, and clears the slice again.  Two accumulation precisions:
//   ACC = F32  (v_mfma_f32_32x32x2_f32, 8 per tile and batch): float32
//              products, two Gaussians per step in list order; for every
//              coefficient map and every float32 decode, so that a map and a
//              decode of it match the fused kernel bit for bit;
//   ACC = BF16 (v_mfma_f32_32x32x16_bf16, 1 per tile and batch): e and w_hat
//              rounded to bfloat16, for BF16 / FP8 decodes of 1024 features
//              without a map (narrower ones take k_render_mx, further down).
// Accumulation is float32 either way, in a fixed order (bit-reproducible).
// After the list the rows go out as the coefficient map (32 pixels at a time
// through LDS, 16-byte pieces of whole rows, float32 / bfloat16 / FP8 E4M3)
// and / or are written to LDS in the decode's precision and decoded on MFMA,
// F^T = C^T W^T, in passes of up to 512 features that leave through LDS as
// 16-byte row pieces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kRB = 16;                 // Gaussians per batch
constexpr int kRKMax = 16;              // Top-K slots per Gaussian
constexpr int kRThreads = 256;          // four waves
constexpr int kRCtrl = 64;              // control words at the end of the LDS block
constexpr int kNoDecode = -1;
constexpr int kBRow = 24;               // bfloat16 per E^T / What^T row: 16 + 8 (conflict-free 16-byte reads)
constexpr int kFRow = 17;               // float32 per What^T row: 16 + 1 (conflict-free 4-byte reads)

__host__ __device__ constexpr int round32(int m) { return (m + 31) / 32 * 32; }
__host__ __device__ constexpr int es_of(int t) { return t == SCOUP_F32 ? 4 : t == SCOUP_BF16 ? 2 : 1; }

// LDS of the list phase (bytes): E (F32: [2][kRB][64] floats; BF16: [2][64][kBRow]) |
// the four waves' What^T slices | code atoms [2][kRB kRKMax] | code values
__host__ __device__ constexpr size_t r_e_bytes(int acc) { return acc == SCOUP_F32 ? 4 * 2 * kRB * 64 : 2 * 2 * 64 * kBRow; }
__host__ __device__ constexpr size_t r_wh_bytes(int acc, int tpw) {
  return acc == SCOUP_F32 ? (size_t)4 * 4 * tpw * 32 * kFRow : (size_t)2 * 4 * tpw * 32 * kBRow;
}
__host__ __device__ constexpr size_t r_region_a(int acc, int tpw) {
  return r_e_bytes(acc) + r_wh_bytes(acc, tpw) + 2 * 4 * 2 * kRB * kRKMax;
}
// bytes per pixel row of W in the decode's precision (16-byte aligned for
// BF16 / FP8; an odd float count for float32): the decode's k range and every
// atom of the 32-atom tiles, plus padding against bank conflicts
__host__ __device__ constexpr int r_wrow(int kpad, int m, int in_t) {
  return in_t == SCOUP_F32 ? ((kpad > round32(m) ? kpad : round32(m)) + 1) * 4
       : in_t == SCOUP_BF16 ? ((kpad > round32(m) ? kpad : round32(m)) + 8) * 2
                            : (kpad > round32(m) ? kpad : round32(m)) + 16;
}
__host__ __device__ constexpr size_t r_w_bytes(int kpad, int m, int in_t) {
  return (64 * (size_t)r_wrow(kpad, m, in_t) + 15) & ~(size_t)15;
}
// column tiles per wave and pass of the decode (a pass covers 4 x 32 features
// per tile), up to four for a float32 decode (its long k loop amortises the
// row reads) and two otherwise.  When one pass covers every feature its
// staging reuses W's LDS; otherwise the staging sits beside W and the pass
// is made as wide as fits.
__host__ __device__ constexpr int r_nch_max(int in_t) { return in_t == SCOUP_F32 ? 4 : 2; }
__host__ __device__ constexpr bool r_pass_fits(int cols, int m, int in_t, int kpad, int out_t) {
  return r_w_bytes(kpad, m, in_t) + (size_t)32 * (cols * es_of(out_t) + 16) + kRCtrl <= 160 * 1024;
}
__host__ __device__ constexpr int r_nch(int npad, int m, int in_t, int kpad, int out_t) {
  return npad / 128 <= r_nch_max(in_t) ? npad / 128
       : (r_nch_max(in_t) >= 4 && r_pass_fits(512, m, in_t, kpad, out_t)) ? 4
       : r_pass_fits(256, m, in_t, kpad, out_t) ? 2 : 1;
}
__host__ __device__ constexpr size_t r_decode_bytes(int m, int in_t, int kpad, int npad, int out_t) {
  return r_nch(npad, m, in_t, kpad, out_t) == npad / 128
             ? std::max(r_w_bytes(kpad, m, in_t), (size_t)32 * (npad * es_of(out_t) + 16))
             : r_w_bytes(kpad, m, in_t) + (size_t)32 * (4 * r_nch(npad, m, in_t, kpad, out_t) * 32 * es_of(out_t) + 16);
}
__host__ __device__ constexpr int r_map_srow(int m, int map_t) { return round32(m) * es_of(map_t) + 16; }
// LDS after the list: the map's staging (32 pixel rows), or W in the decode's
// precision followed by the staging of one pass of features (32 pixel rows)
__host__ __device__ constexpr size_t r_region_b(int m, bool map, int map_t, int in_t, int kpad, int npad, int out_t) {
  return std::max(map ? (size_t)32 * r_map_srow(m, map_t) : (size_t)0,
                  in_t == kNoDecode ? (size_t)0 : r_decode_bytes(m, in_t, kpad, npad, out_t));
}
__host__ __device__ constexpr int r_tpw(int m) { return (round32(m) / 32 + 3) / 4 <= 1 ? 1 : (round32(m) / 32 + 3) / 4 <= 2 ? 2 : 4; }

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
  // format 0 = FP8 E4M3 for both operands; E8M0 block scales 127 = 2^0
  static __device__ __forceinline__ f16v mfma(i32x8 a, i32x8 b, f16v c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
};

// four consecutive values into memory in a storage type (16, 8 or 4 bytes)
__device__ __forceinline__ void put4(uint8_t* p, int t, float a, float b, float c, float d) {
  if (t == SCOUP_F32) {
    *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
  } else if (t == SCOUP_BF16) {
    const unsigned int lo = f32x2_to_bf16(a, b);
    const unsigned int hi = f32x2_to_bf16(c, d);
    *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi);
  } else {
    *reinterpret_cast<unsigned int*>(p) = f32x4_to_e4m3(a, b, c, d);
  }
}

// `rows` pixel rows staged in LDS (stride srow) -> the image: `bytes` per
// pixel at byte row_off of a record of rec bytes; 16-byte pieces where aligned
__device__ __forceinline__ void store_rows(uint8_t* dst, const uint8_t* stage, int srow, int p0, int rows,
                                           int bytes, long long rec, long long row_off, int tile_x0, int tile_y0,
                                           int Wd, int Hd, int tid) {
  const bool vec = (bytes & 15) == 0 && (rec & 15) == 0 && (row_off & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
  if (vec) {
    const int pieces = bytes / 16;
    for (int c = tid; c < rows * pieces; c += kRThreads) {
      const int r = c / pieces, q = c - r * pieces;
      const int p = p0 + r;
      const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
      if (ox >= Wd || oy >= Hd) continue;
      *reinterpret_cast<i32x4*>(dst + ((long long)oy * Wd + ox) * rec + row_off + q * 16) =
          *reinterpret_cast<const i32x4*>(stage + r * srow + q * 16);
    }
  } else {
    for (int c = tid; c < rows * bytes; c += kRThreads) {
      const int r = c / bytes, b = c - r * bytes;
      const int p = p0 + r;
      const int ox = tile_x0 + (p & 7), oy = tile_y0 + (p >> 3);
      if (ox >= Wd || oy >= Hd) continue;
      dst[((long long)oy * Wd + ox) * rec + row_off + b] = stage[r * srow + b];
    }
  }
}

// three workgroups per CU (at most 168 registers) for the map alone at up to
// 256 atoms; two otherwise (a decode's W and staging leave LDS for two
// workgroups anyway, so a tighter register bound would only spill)
template <int ACC, int IN_T, int TPW>
struct RWpe {
  static constexpr int v = (TPW <= 2 && IN_T == kNoDecode) ? 3 : 2;
};

template <int ACC, int IN_T, int TPW>
__global__ __launch_bounds__(kRThreads) __attribute__((amdgpu_waves_per_eu(RWpe<ACC, IN_T, TPW>::v))) void
k_render(const RenderBlockArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const BinArgs& bn = a.bin;
  Status* st = bn.status;
  if (st->view_overflow) return;
  const int M = a.m_atoms, K = a.k;
  const size_t ra = r_region_a(ACC, TPW);
  const size_t rb = r_region_b(M, a.map != nullptr, a.map_dtype, IN_T, a.kpad, a.npad, a.out_dtype);
  uint8_t* E8 = lds;                                                      // E, double buffered
  uint8_t* Wh8 = lds + r_e_bytes(ACC);                                    // What^T slices
  int* CI = reinterpret_cast<int*>(Wh8 + r_wh_bytes(ACC, TPW));          // [2][kRB * kRKMax]
  float* CV = reinterpret_cast<float*>(CI + 2 * kRB * kRKMax);
  int* ctrl = reinterpret_cast<int*>(lds + std::max(ra, rb));           // live[2], n_batches (ordered by barriers)

  const int tile = (int)bn.tile_order[blockIdx.x];                       // longest lists first
  const int tx = tile % bn.tiles_x, ty = tile / bn.tiles_x;
  const int Wd = bn.cam.width, Hd = bn.cam.height;
  const unsigned int start = bn.tile_start[tile];
  const int L = (int)(bn.tile_start[tile + 1] - start);
  const unsigned long long* keys = bn.keys[bn.sorted];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tile_x0 = tx * 8, tile_y0 = ty * 8;
  const int ntiles = round32(M) / 32;               // 32-atom tiles; wave w owns w, w+4, ...
  float* whf = reinterpret_cast<float*>(Wh8) + wave * TPW * 32 * kFRow;         // F32: [TPW*32][kFRow]
  uint16_t* whb = reinterpret_cast<uint16_t*>(Wh8) + wave * TPW * 32 * kBRow;   // BF16: [TPW*32][kBRow]
  if (ACC == SCOUP_F32)
    for (int j = lane; j < TPW * 32 * kFRow; j += 64) whf[j] = 0.0f;
  else
    for (int j = lane; j < TPW * 32 * kBRow; j += 64) whb[j] = 0;
  const int nb_total = (L + kRB - 1) / kRB;
  if (tid == 0) ctrl[2] = nb_total;
  __syncthreads();

  f16v acc[TPW][2];
#pragma unroll
  for (int t = 0; t < TPW; ++t) { acc[t][0] = (f16v){}; acc[t][1] = (f16v){}; }

  const int lx = lane & 7, ly = lane >> 3;
  const bool inside = tile_x0 + lx < Wd && tile_y0 + ly < Hd;
  float T = inside ? 1.0f : -1.0f;                 // wave 0: transmittance, negated once finished
  unsigned int count = 0u;
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  const int nslots = kRB * K;
  // wave 0 prefetch: ids two batches ahead, splats and code slots one batch
  // ahead (lanes < kRB hold a batch's ids and splats; lane t holds code slot
  // t mod K of Gaussian t / K)
  auto key_at = [&](int i) { return (unsigned int)keys[start + min(i, max(L - 1, 0))]; };
  auto load_data = [&](unsigned int key, GSplat& sp, int (&ci)[4], float (&cv)[4]) {
    if (lane < kRB) sp = bn.splats[key];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = min(lane + 64 * r, nslots - 1);
      const int g = t / K, s = t - g * K;
      const unsigned int id = (unsigned int)__shfl((int)key, g, 64);
      // 32-bit byte offsets from the arrays' uniform bases (n k < 2^30, checked
      // on the host): no per-lane 64-bit addresses to keep across the loop
      const unsigned int off = (id * (unsigned int)K + (unsigned int)s) * 4u;
      ci[r] = *reinterpret_cast<const int*>(reinterpret_cast<const uint8_t*>(a.topk_idx) + off);
      cv[r] = *reinterpret_cast<const float*>(reinterpret_cast<const uint8_t*>(a.topk_val) + off);
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

  // ---- the list: composite (wave 0), accumulate (every wave) ------------------
  int nb_run = nb_total;
  for (int it = 0; it <= nb_run; ++it) {
    const int buf = it & 1;
    if (wave == 0 && it < nb_run) {
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
      GSplat sp1;
      int ci1[4];
      float cv1[4];
      const bool more = b0 + kRB < L;
      unsigned int key2 = key1;
      if (more) {                                    // loads of the next batches in flight during this one
        load_data(key1, sp1, ci1, cv1);
        key2 = key_at(b0 + 2 * kRB + (lane & (kRB - 1)));
      }
      unsigned int kept = 0u, ep[kRB / 2];
      float* ef = reinterpret_cast<float*>(E8) + buf * kRB * 64;
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
        if (ACC == SCOUP_F32) {
          ef[g * 64 + lane] = e;
        } else {
          const unsigned int eb = f32_to_bf16_rne(e);
          if (g & 1) ep[g >> 1] |= eb << 16; else ep[g >> 1] = eb;
        }
      }
      if (ACC == SCOUP_BF16) {                        // this pixel's row of E^T: two 16-byte stores
        uint4* erow = reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(E8) + (buf * 64 + lane) * kBRow);
        erow[0] = make_uint4(ep[0], ep[1], ep[2], ep[3]);
        erow[1] = make_uint4(ep[4], ep[5], ep[6], ep[7]);
      }
      count += (unsigned int)__popc(kept);
      unsigned int live = kept;                        // Gaussians with a contribution in the block
      for (int o = 32; o >= 1; o >>= 1) live |= (unsigned int)__shfl_xor((int)live, o, 64);
      const bool finished = __ballot(T > 0.0f) == 0ull;   // every pixel of the block
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
      // batch it-1: this wave's code slots into its What^T slice, the MFMAs,
      // the slice cleared again
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
            const int row = ((j >> 5) >> 2) * 32 + (j & 31);
            if (ACC == SCOUP_F32) {
              slot[r] = row * kFRow + g;
              whf[slot[r]] = cv[t];
            } else {
              slot[r] = row * kBRow + g;
              whb[slot[r]] = f32_to_bf16_rne(cv[t]);
            }
          }
        }
      }
      if (ACC == SCOUP_F32) {
        const float* eb = reinterpret_cast<const float*>(E8) + pb * kRB * 64;
#pragma unroll
        for (int s = 0; s < kRB / 2; ++s) {
          const int g = 2 * s + (lane >> 5);
          const float b0 = eb[g * 64 + (lane & 31)], b1 = eb[g * 64 + 32 + (lane & 31)];
#pragma unroll
          for (int t = 0; t < TPW; ++t) {
            if (wave + 4 * t >= ntiles) break;
            const float av = whf[(t * 32 + (lane & 31)) * kFRow + g];
            acc[t][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b0, acc[t][0], 0, 0, 0);
            acc[t][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b1, acc[t][1], 0, 0, 0);
          }
        }
      } else {
        const uint16_t* eb = reinterpret_cast<const uint16_t*>(E8) + pb * 64 * kBRow;
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          if (wave + 4 * t >= ntiles) break;
          const bf16x8 A = *reinterpret_cast<const bf16x8*>(whb + (t * 32 + (lane & 31)) * kBRow + 8 * (lane >> 5));
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bf16x8 B = *reinterpret_cast<const bf16x8*>(eb + (h * 32 + (lane & 31)) * kBRow + 8 * (lane >> 5));
            acc[t][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[t][h], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (slot[r] >= 0) {
          if (ACC == SCOUP_F32) whf[slot[r]] = 0.0f; else whb[slot[r]] = 0;
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
  // accumulator element r of lane l in tile (wave + 4t, half h): pixel h 32 + l % 32,
  // atom 32 (wave + 4t) + 8 (r / 4) + 4 (l / 32) + r % 4

  // ---- the coefficient map: 32 pixel rows at a time through LDS ----------------
  if (a.map) {
    const int mes = es_of(a.map_dtype);
    const int srow = r_map_srow(M, a.map_dtype);
    const float sc = a.map_scale;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint8_t* row = lds + (lane & 31) * srow;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tl = wave + 4 * t;
        if (tl >= ntiles) break;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j0 = tl * 32 + 8 * q + 4 * (lane >> 5);
          const f16v& v = acc[t][h];
          put4(row + j0 * mes, a.map_dtype, v[4 * q] * sc, v[4 * q + 1] * sc, v[4 * q + 2] * sc, v[4 * q + 3] * sc);
        }
      }
      __syncthreads();
      store_rows(reinterpret_cast<uint8_t*>(a.map), lds, srow, h * 32, 32, M * mes, (long long)M * mes, 0, tile_x0,
                 tile_y0, Wd, Hd, tid);
      __syncthreads();
    }
  }

  // ---- the decode F^T = C^T W^T on MFMA -------------------------------------------
  if constexpr (IN_T != kNoDecode) {
    using FR = RFrag<IN_T>;
    using FT = typename FR::type;
    constexpr int es = es_of(IN_T);
    const int wrow = r_wrow(a.kpad, M, IN_T);
    uint8_t* Wq = lds;                                // W in the decode's precision, pixel rows
    const float qs = IN_T == SCOUP_FP8_E4M3 ? a.q_scale : 1.0f;
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
          if (IN_T == SCOUP_F32) {                   // rows of an odd float count: four 4-byte stores
            float* w = reinterpret_cast<float*>(Wq + p * wrow) + j0;
            w[0] = v[4 * q]; w[1] = v[4 * q + 1]; w[2] = v[4 * q + 2]; w[3] = v[4 * q + 3];
          } else {
            put4(Wq + p * wrow + j0 * es, IN_T, v[4 * q] * qs, v[4 * q + 1] * qs, v[4 * q + 2] * qs,
                 v[4 * q + 3] * qs);
          }
        }
      }
    }
    const int kz = a.kpad - ntiles * 32;            // the decode's k padding past the tiles: zero
    for (int c = tid; c < 64 * kz * es; c += kRThreads) {
      const int p = c / (kz * es), b = c - p * (kz * es);
      Wq[p * wrow + ntiles * 32 * es + b] = 0;
    }
    __syncthreads();

    const int nks = a.kpad / FR::KS;
    const FT* Bf = reinterpret_cast<const FT*>(a.codebook_prep);
    float mul = a.out_mul;
    if (a.cb_scale) mul /= *a.cb_scale;
    const int OES = es_of(a.out_dtype);
    const int D = a.d;
    // passes of NCH column tiles per wave (two live accumulators per pixel
    // half): pass ps, wave w owns tiles (4 ps + w) NCH + c, so a pass covers
    // 4 NCH x 32 consecutive features, staged 32 pixels at a time (over W
    // when one pass covers all of them, past W's rows otherwise)
    const int nct = a.npad / 128;                    // column tiles per wave over all passes
    const int nch = r_nch(a.npad, M, IN_T, a.kpad, a.out_dtype);
    const bool over = nch == nct;
    uint8_t* stage = over ? lds : lds + r_w_bytes(a.kpad, M, IN_T);
    auto passes = [&](auto nch_c) {
      constexpr int NCH = decltype(nch_c)::value;
      constexpr int pcols = 4 * NCH * 32;
      const int srow = pcols * OES + 16;
      for (int ps = 0; ps < nct / NCH; ++ps) {
        const int ct0 = (4 * ps + wave) * NCH;
        f16v fo[2][NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) fo[0][c] = fo[1][c] = (f16v){};
        auto load_b = [&](FT (&b)[NCH], int ks) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) b[c] = Bf[((long long)(ct0 + c) * nks + ks) * 64 + lane];
        };
        auto mma = [&](const FT (&b)[NCH], int ks) {
          FT af[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int p = h * 32 + (lane & 31);
            af[h] = *reinterpret_cast<const FT*>(Wq + p * wrow + (ks * FR::KS + (lane >> 5) * (FR::KS / 2)) * es);
          }
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            fo[0][c] = FR::mfma(b[c], af[0], fo[0][c]);
            fo[1][c] = FR::mfma(b[c], af[1], fo[1][c]);
          }
        };
        if ((nks & 1) == 0) {
          // codebook fragments one k-step ahead in two register sets that
          // alternate (no copies, so no wait at the loop's end); each set is
          // loaded right after its last use, the loads pinned there
          FT b0[NCH], b1[NCH];
          load_b(b0, 0);
          for (int ks = 0; ks < nks; ks += 2) {
            load_b(b1, ks + 1);
            asm volatile("" ::: "memory");
            mma(b0, ks);
            load_b(b0, min(ks + 2, nks - 1));       // the last pass reloads a fragment it does not use
            asm volatile("" ::: "memory");
            mma(b1, ks + 1);
          }
        } else {
          FT bcur[NCH], bnext[NCH];
          load_b(bcur, 0);
          for (int ks = 0; ks < nks; ++ks) {
            if (ks + 1 < nks) load_b(bnext, ks + 1);
            mma(bcur, ks);
            if (ks + 1 < nks) {
#pragma unroll
              for (int c = 0; c < NCH; ++c) bcur[c] = bnext[c];
            }
          }
        }
        if (over) __syncthreads();                   // every wave has read W: its LDS now stages features
        const int col0 = ps * pcols;                 // first feature of the pass
        const int ncol = min(pcols, D - col0);       // its columns inside D
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          uint8_t* row = stage + (lane & 31) * srow;
#pragma unroll
          for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
              const int d0 = (wave * NCH + c) * 32 + 8 * rg + 4 * (lane >> 5);   // column within the pass
              const f16v& v = fo[h][c];
              put4(row + d0 * OES, a.out_dtype, v[4 * rg] * mul, v[4 * rg + 1] * mul, v[4 * rg + 2] * mul,
                   v[4 * rg + 3] * mul);
            }
          __syncthreads();
          if (ncol > 0)
            store_rows(reinterpret_cast<uint8_t*>(a.features), stage, srow, h * 32, 32, ncol * OES,
                       (long long)D * OES, (long long)col0 * OES, tile_x0, tile_y0, Wd, Hd, tid);
          __syncthreads();
        }
      }
    };
    if constexpr (r_nch_max(IN_T) >= 4) {
      if (nch == 4) { passes(std::integral_constant<int, 4>{}); return; }
    }
    if (nch == 2) passes(std::integral_constant<int, 2>{});
    else passes(std::integral_constant<int, 1>{});
  }
}

// four outputs into LDS (float32: 16 bytes, bfloat16: 8 bytes)
__device__ __forceinline__ void lds_store4(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ void lds_store4(uint16_t* p, float a, float b, float c, float d) {
  const unsigned int lo = f32x2_to_bf16(a, b);
  const unsigned int hi = f32x2_to_bf16(c, d);
  *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi);
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
// decode's precision and the block is decoded as in k_render.  (With its
// column passes fixed at compile time it runs faster than k_render's ACC =
// BF16 instance, which serves only 1024-feature decodes.)
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

// three workgroups per CU (at most 168 registers) for BF16 and FP8 up to 256
// atoms; two otherwise
template <int IN_T, int NCT, int TPW, int WPE = (TPW <= 2 ? 3 : 2)>
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
      // 32-bit byte offsets from the arrays' uniform bases (n k < 2^30, checked
      // on the host): no per-lane 64-bit addresses to keep across the loop
      const unsigned int off = (id * (unsigned int)K + (unsigned int)s) * 4u;
      ci[r] = *reinterpret_cast<const int*>(reinterpret_cast<const uint8_t*>(a.topk_idx) + off);
      cv[r] = *reinterpret_cast<const float*>(reinterpret_cast<const uint8_t*>(a.topk_val) + off);
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
          const unsigned int lo = f32x2_to_bf16(v[4 * q], v[4 * q + 1]);
          const unsigned int hi = f32x2_to_bf16(v[4 * q + 2], v[4 * q + 3]);
          *reinterpret_cast<uint2*>(Wq + p * wrow + 2 * j0) = make_uint2(lo, hi);
        } else {
          const unsigned int w4 = f32x4_to_e4m3(v[4 * q] * a.q_scale, v[4 * q + 1] * a.q_scale,
                                                v[4 * q + 2] * a.q_scale, v[4 * q + 3] * a.q_scale);
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
    auto load_b = [&](FT (&b)[NCH], int ks) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) b[c] = Bf[((long long)(ct0 + c) * nks + ks) * 64 + lane];
    };
    auto mma = [&](const FT (&b)[NCH], int ks) {
      FT af[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = h * 32 + (lane & 31);
        af[h] = *reinterpret_cast<const FT*>(Wq + p * wrow + (ks * FR::KS + (lane >> 5) * (FR::KS / 2)) * es);
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        fo[0][c] = FR::mfma(b[c], af[0], fo[0][c]);
        fo[1][c] = FR::mfma(b[c], af[1], fo[1][c]);
      }
    };
    if ((nks & 1) == 0) {                        // alternating register sets (as in k_render)
      FT b0[NCH], b1[NCH];
      load_b(b0, 0);
      for (int ks = 0; ks < nks; ks += 2) {
        load_b(b1, ks + 1);
        asm volatile("" ::: "memory");
        mma(b0, ks);
        load_b(b0, min(ks + 2, nks - 1));
        asm volatile("" ::: "memory");
        mma(b1, ks + 1);
      }
    } else {
      FT bcur[NCH], bnext[NCH];
      load_b(bcur, 0);
      for (int ks = 0; ks < nks; ++ks) {
        if (ks + 1 < nks) load_b(bnext, ks + 1);
        mma(bcur, ks);
        if (ks + 1 < nks) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) bcur[c] = bnext[c];
        }
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


// BF16 / FP8 decodes without a map take bfloat16 products; everything else float32
static int render_acc(const RenderBlockArgs& a) {
  return ((a.in_dtype == SCOUP_BF16 || a.in_dtype == SCOUP_FP8_E4M3) && !a.map) ? SCOUP_BF16 : SCOUP_F32;
}

size_t render_block_lds_bytes(const RenderBlockArgs& a) {
  return std::max(r_region_a(render_acc(a), r_tpw(a.m_atoms)),
                  r_region_b(a.m_atoms, a.map != nullptr, a.map_dtype, a.in_dtype, a.kpad, a.npad, a.out_dtype)) +
         kRCtrl;
}

template <int ACC, int IN_T>
static void launch_r(const RenderBlockArgs& a, hipStream_t s) {
  const size_t lds = render_block_lds_bytes(a);
  switch (r_tpw(a.m_atoms)) {
    case 1: hipLaunchKernelGGL((k_render<ACC, IN_T, 1>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_render<ACC, IN_T, 2>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a); break;
    default: hipLaunchKernelGGL((k_render<ACC, IN_T, 4>), dim3(a.bin.n_tiles), dim3(kRThreads), lds, s, a); break;
  }
}

hipError_t launch_render_block(RenderBlockArgs& a, hipStream_t s, int stage) {
  if (a.k < 1 || a.k > kRKMax || a.m_atoms < 1 || a.m_atoms > 512) return hipErrorInvalidValue;
  if (a.in_dtype != kNoDecode) {
    const int nct = a.npad / 128;
    if (nct != 1 && nct != 2 && nct != 4 && nct != 8) return hipErrorInvalidValue;
  }
  hipError_t e = launch_bin_view(a.bin, s);
  if (e != hipSuccess) return e;
  if (a.bin.n_tiles == 0) return hipSuccess;
  StageTimer::begin(stage, s);
  const bool bf = render_acc(a) == SCOUP_BF16;
  if (bf && a.npad <= 512) {
    e = a.in_dtype == SCOUP_BF16 ? launch_mx<SCOUP_BF16>(a, s) : launch_mx<SCOUP_FP8_E4M3>(a, s);
    StageTimer::end(stage, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  switch (a.in_dtype) {
    case SCOUP_F32: launch_r<SCOUP_F32, SCOUP_F32>(a, s); break;
    case SCOUP_BF16:
      if (bf) launch_r<SCOUP_BF16, SCOUP_BF16>(a, s); else launch_r<SCOUP_F32, SCOUP_BF16>(a, s);
      break;
    case SCOUP_FP8_E4M3:
      if (bf) launch_r<SCOUP_BF16, SCOUP_FP8_E4M3>(a, s); else launch_r<SCOUP_F32, SCOUP_FP8_E4M3>(a, s);
      break;
    default: launch_r<SCOUP_F32, kNoDecode>(a, s); break;
  }
  StageTimer::end(stage, s);
  return hipGetLastError();
}

template <int ACC, int IN_T>
static hipError_t set_r_lds() {
  const auto attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  const int lim = 160 * 1024;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_render<ACC, IN_T, 1>, attr, lim)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_render<ACC, IN_T, 2>, attr, lim)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_render<ACC, IN_T, 4>, attr, lim);
}

hipError_t render_set_lds_limits() {
  hipError_t e;
  if ((e = set_mx_lds_all<SCOUP_BF16>()) != hipSuccess) return e;
  if ((e = set_mx_lds_all<SCOUP_FP8_E4M3>()) != hipSuccess) return e;
  if ((e = set_r_lds<SCOUP_F32, kNoDecode>()) != hipSuccess) return e;
  if ((e = set_r_lds<SCOUP_F32, SCOUP_F32>()) != hipSuccess) return e;
  if ((e = set_r_lds<SCOUP_F32, SCOUP_BF16>()) != hipSuccess) return e;
  if ((e = set_r_lds<SCOUP_F32, SCOUP_FP8_E4M3>()) != hipSuccess) return e;
  if ((e = set_r_lds<SCOUP_BF16, SCOUP_BF16>()) != hipSuccess) return e;
  return set_r_lds<SCOUP_BF16, SCOUP_FP8_E4M3>();
}

}  // namespace scoup
