// Uplift path of libscoup: front-to-back compositing fused with the weighted
// sparse accumulation, the per-Gaussian row build across views, and Top-K.
// gfx950 (CDNA4), wave64.
//
// Paper mapping:
//   k_composite_blk  Eq. 2 weights e = alpha T on one 8x8 block, reduced per
//                    (Gaussian, block region) -- the pixels of a region share one
//                    code (Sec. 4.1), so Algorithm 1's inner loop collapses to
//                    one weight per (Gaussian, region) touch.  The first two
//                    regions of a block go to fixed record slots of the
//                    (Gaussian, block) pair; further regions become deferred
//                    entries added to the accumulator after the view.
//   k_rowbuild       Eq. 5 / Algorithm 1: w_i[j] += c_j * weight for every
//                    record of Gaussian i over a batch of views, in LDS; rows
//                    written once, coalesced; Eq. 6 Top-K fused on the last batch.
//   k_topk           Eq. 6 on an accumulator in memory.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {


// ---------------------------------------------------------------------------
// composite + per-(Gaussian, block, region) reduction: one 8x8 pixel block per
// workgroup (one wave), lane l = pixel (l & 7, l >> 3) of the block, the
// block's list already in depth order (binning).
// Per batch of 32 depth-ordered Gaussians the wave writes every pixel's
// weight e into an LDS matrix E[Gaussian][pixel] (no cross-lane traffic
// inside the sequential compositing loop).  The batch's weight per
// (Gaussian, region) is then the product of E with the block's 0/1 pixel-
// membership matrix M[pixel][column], a dense contraction over the 64 pixels
// done on the matrix cores (MFMA 16x16x4 f32: two tiles of 16 Gaussians by
// 16 columns).  Columns 2l and 2l + 1 are level l's two record regions of
// the block (the (Gaussian, block) pair's record slots); the columns after
// them are further regions of the block, whose weights become deferred
// entries that k_apply_extra adds to the accumulator after the view.
// Regions beyond the 16 columns (blocks cut into many regions) are reduced
// with a per-region loop over E.
// ---------------------------------------------------------------------------
constexpr int kEStride = 68;                 // 64 pixels + 4: rows 16-byte aligned, b128 reads conflict-free
constexpr int kCompositeBatch = 32;          // Gaussians per batch: 16-row MFMA tiles
constexpr int kCompositeWaves = 4;           // waves per SIMD the register budget allows
constexpr int kCols = 16;                    // membership columns (one MFMA tile)

typedef float f4v __attribute__((ext_vector_type(4)));

// Adds w times region greg's code (or feature, for the dense uplift) to
// Gaussian id's accumulator row of level view lv.
__device__ __forceinline__ void add_region_direct(const int* code_idx, const float* code_val, int k_code,
                                                  const float* dense_F, int dense_d, float* acc, float* zsum,
                                                  unsigned int id, long long greg, float w, int m_atoms,
                                                  Status* st) {
  atomicAdd(&st->n_direct, 1ull);
  if (dense_F) {
    const long long fr = greg * dense_d;
    const unsigned long long drow = (unsigned long long)id * (unsigned long long)dense_d;
    for (int c = 0; c < dense_d; ++c) atomic_add_f32(&acc[drow + c], w * dense_F[fr + c]);
    atomic_add_f32(&zsum[id], w);
  } else {
    const long long gr = greg * k_code;
    const unsigned long long arow = (unsigned long long)id * (unsigned long long)m_atoms;
    for (int c = 0; c < k_code; ++c) {
      const int jj = code_idx[gr + c];
      if (jj >= m_atoms) atomicOr(&st->data_error, 2u);
      else if (jj >= 0) atomic_add_f32(&acc[arow + (unsigned long long)jj], w * code_val[gr + c]);
    }
  }
}

template <int B, int WPE, int NL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_composite_blk(
    const GSplat* __restrict__ splats, const unsigned int* __restrict__ tile_start,
    const unsigned int* __restrict__ order,
    const unsigned long long* __restrict__ keys, int tiles_x, int W,
    int H, int n_levels, int m_atoms, UpliftViewArgs args, Status* st) {
  constexpr int NT = B / 16;                   // 16-Gaussian MFMA tiles per batch
  __shared__ __align__(16) float E[B * kEStride];
  __shared__ float4 s_bs[2 * (B + 2)];         // the batch's splats, block-relative: (hx, hy, fx, fy),
  __shared__ float s_q[B + 2];                 //   (l00, l10, l11, opacity) and qmax; two spare slots
                                               //   for the reads one step ahead
  __shared__ __align__(16) unsigned int s_pidx[B];   // the batch Gaussians' pair (record) indices
  __shared__ __align__(16) unsigned int s_gid[B];    // and ids
  __shared__ unsigned long long s_excl[kMaxLevels];  // per level: pixels whose region has a column
  if (st->view_overflow) return;
  if (NL == 1) n_levels = 1;                   // one-level instance: the per-level loops fold away
  const int tile = (int)order[blockIdx.x];      // longest lists first
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const unsigned int start = tile_start[tile];
  const int L = (int)(tile_start[tile + 1] - start);
  const int lane = threadIdx.x;
  // lanes 16 q .. 16 q + 15 hold the 4x4 quadrant q of the block (every
  // per-pixel mask below is a ballot over lanes, so the order is free)
  const int qd = lane >> 4, qi = lane & 15;
  const int lx = (qd & 1) * 4 + (qi & 3), ly = (qd >> 1) * 4 + (qi >> 2);
  const int tile_x0 = tx * 8, tile_y0 = ty * 8;
  const int px = tile_x0 + lx, py = tile_y0 + ly;
  const bool inside = px < W && py < H;
  // Per level: the pixel's region (validated on every pixel, empty blocks
  // included); record regions r0 = region of the first pixel with one, r1 =
  // first other region; then one column per further region while columns
  // last.  Column masks and (level, global region) go through LDS (E's space,
  // unused before the first batch).
  unsigned long long* s_cm = reinterpret_cast<unsigned long long*>(E);   // [kCols] pixel masks
  int* s_ci = reinterpret_cast<int*>(E + 2 * kCols);                    // [kCols][2] level, region
  int regs[NL];                        // the pixel's region per level (-1: none or invalid)
  int ncols = 2 * n_levels;
  unsigned int spill = 0u;                     // bit l: level l has regions without a column
  int rg0[NL], rg1[NL];        // per level: global ids of the two record regions (-1: none)
  int pkey = 0;                                // bits 2l, 2l+1: the pixel's record slot at level l (2: none)
  bool pvalid = false;                         // the pixel is in some record region
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    regs[l] = -1;
    rg0[l] = -1; rg1[l] = -1;
    if (l >= n_levels) continue;
    const LevelView& lv = args.lv[l];
    int reg = -1;
    if (inside) {
      reg = lv.rmap[(long long)py * W + px];
      if (reg < -1 || reg >= lv.n_regions) { atomicOr(&st->data_error, 1u); reg = -1; }
    }
    regs[l] = reg;
    const unsigned long long any = __ballot(reg >= 0);
    const int r0 = any ? __builtin_amdgcn_readlane(reg, __ffsll((long long)any) - 1) : -1;
    const unsigned long long oth = __ballot(reg >= 0 && reg != r0);
    const int r1 = oth ? __builtin_amdgcn_readlane(reg, __ffsll((long long)oth) - 1) : -1;
    const unsigned long long m0 = __ballot(reg >= 0 && reg == r0);
    const unsigned long long m1 = __ballot(reg >= 0 && reg == r1);
    rg0[l] = r0 >= 0 ? (int)(lv.region_base + r0) : -1;
    rg1[l] = r1 >= 0 ? (int)(lv.region_base + r1) : -1;
    if (lane == 0) {
      s_cm[2 * l] = m0; s_cm[2 * l + 1] = m1;
      s_ci[4 * l] = l; s_ci[4 * l + 1] = rg0[l];
      s_ci[4 * l + 2] = l; s_ci[4 * l + 3] = rg1[l];
    }
    const int code = (reg >= 0 && reg == r0) ? 0 : ((reg >= 0 && reg == r1) ? 1 : 2);
    pkey |= code << (2 * l);
    pvalid = pvalid || code < 2;
    unsigned long long covered = m0 | m1;
    unsigned long long rest = __ballot(reg >= 0) & ~covered;
    while (rest && ncols < kCols) {
      const int rr = __builtin_amdgcn_readlane(reg, __ffsll((long long)rest) - 1);
      const unsigned long long m = __ballot(reg == rr);
      rest &= ~m;
      covered |= m;
      if (lane == 0) { s_cm[ncols] = m; s_ci[2 * ncols] = l; s_ci[2 * ncols + 1] = (int)(lv.region_base + rr); }
      ++ncols;
    }
    if (rest) spill |= 1u << l;
    if (lane == 0) s_excl[l] = covered;
  }
  for (int l = n_levels; l < kMaxLevels; ++l) pkey |= 2 << (2 * l);
  if (L == 0) return;
  // Pixel classes (same record slot at every level).  With no further
  // regions and at most two classes, the reduction is two masked row sums
  // of E per Gaussian (the common case); otherwise the MFMA product.
  const unsigned long long vmask = __ballot(pvalid);
  const int key0 = vmask ? __builtin_amdgcn_readlane(pkey, __ffsll((long long)vmask) - 1) : 0;
  const unsigned long long cm0 = __ballot(pvalid && pkey == key0);
  const unsigned long long rest1 = vmask & ~cm0;
  const int key1 = rest1 ? __builtin_amdgcn_readlane(pkey, __ffsll((long long)rest1) - 1) : 0;
  const unsigned long long cm1 = __ballot(pvalid && pkey == key1) & rest1;
  const bool two_class = ncols == 2 * n_levels && (vmask & ~cm0 & ~cm1) == 0ull;
  const bool full0 = cm0 == ~0ull;             // one class covering the whole block
  // deferred entries of the further-region columns: one slot per (list
  // entry, column), reserved at once (weights of zero included)
  const int n_ext = ncols - 2 * n_levels;
  unsigned long long ebase = 0ull;
  if (n_ext > 0) {
    if (lane == 0) ebase = atomicAdd(&st->n_extra, (unsigned long long)L * (unsigned long long)n_ext);
    ebase = __shfl(ebase, 0, 64);
  }
  __syncthreads();
  // This lane's part of M and of the output: column col, K slot kk (pixels
  // 16 kk .. 16 kk + 15, one per MFMA step), output rows 4 kk .. 4 kk + 3 of
  // each 16-Gaussian tile.
  const int col = lane & 15, kk = lane >> 4;
  const bool rec_col = col < 2 * n_levels;
  const bool ext_col = !rec_col && col < ncols;
  unsigned int mbits = 0u;                     // bit s: M[16 kk + s][col]
  int col_level = -1, col_greg = -1;
  if (col < ncols) {
    mbits = (unsigned int)(s_cm[col] >> (16 * kk)) & 0xFFFFu;
    col_level = s_ci[2 * col];
    col_greg = s_ci[2 * col + 1];
  }
  float2* rec_out = nullptr;
#pragma unroll
  for (int l = 0; l < NL; ++l)
    if (rec_col && (col >> 1) == l) rec_out = args.lv[l].records;
  if (lane == 0) {                             // slot B: a Gaussian never taken (steps past a quadrant's list)
    s_bs[2 * B] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    s_bs[2 * B + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    s_q[B] = -1.0f;
  }
  __syncthreads();                             // column data read before E is overwritten

  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;
  float T = inside ? 1.0f : -1.0f;             // transmittance; negative once the pixel is finished
  unsigned long long count = 0u;               // the block's contributions
  const int gk = lane % B;                     // lane group g holds Gaussian gk of the batch
  const int gq0 = lane - gk;                   // first pixel of the lane's group (per-region loop)
  // the batch's ids and splats arrive ahead of use: the ids two batches
  // ahead and the splats one batch ahead are loaded while a batch composites
  // (indices past the list are clamped to its last entry: the loads stay
  // unconditional, so nothing waits for them before their batch)
  unsigned long long key_cur = keys[start + min(gk, L - 1)];
  unsigned long long key_next = keys[start + min(B + gk, L - 1)];
  GSplat sp_cur = splats[(unsigned int)key_cur];
  unsigned int off_cur = sp_cur.depth_bits;   // the Gaussian's first pair (record) index (binning put it there)
  for (int b0 = 0; b0 < L; b0 += B) {
    const bool all_done = __ballot(T > 0.0f) == 0ull;
    // every pixel finished: the remaining pairs keep their cleared records;
    // only deferred-entry slots (reserved for the whole list) still need zeros
    if (all_done && n_ext == 0) break;
    const int j = b0 + gk;
    const int nb = min(B, L - b0);
    const GSplat sp_next = splats[(unsigned int)key_next];
    const unsigned int off_next = sp_next.depth_bits;
    const unsigned long long key_after = keys[start + min(j + 2 * B, L - 1)];
    unsigned int my_id = 0;
    unsigned int qmask = 0u;                   // lane < B: quadrants of the block Gaussian gk's box reaches
    if (j < L) {
      my_id = (unsigned int)key_cur;
      if (lane < B) {                          // LDS copy read back in the loop
        const GSplat gg = sp_cur;
        const int ex0 = gg.bx0 - tile_x0, ex1 = gg.bx1 - tile_x0, ey0 = gg.by0 - tile_y0, ey1 = gg.by1 - tile_y0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int qx = (q & 1) * 4, qy = (q >> 1) * 4;
          if (ex0 <= qx + 3 && ex1 >= qx && ey0 <= qy + 3 && ey1 >= qy) qmask |= 1u << q;
        }
        BlockSplat bs;
        bs.load(gg, tile_x0, tile_y0);
        s_bs[2 * lane] = make_float4(bs.hx, bs.hy, bs.fx, bs.fy);
        s_bs[2 * lane + 1] = make_float4(bs.l00, bs.l10, bs.l11, bs.opacity);
        s_q[lane] = bs.qmax;
        const int bx0 = gg.bx0 >> 3, bx1 = gg.bx1 >> 3, by0 = gg.by0 >> 3;
        s_pidx[lane] = off_cur + (unsigned int)((ty - by0) * (bx1 - bx0 + 1) + (tx - bx0));
        s_gid[lane] = my_id;
      }
    }
    __syncthreads();
    // Each quadrant steps through the batch Gaussians whose box reaches it, in
    // list order: a Gaussian skipped by a quadrant has alpha < 1/255 at all of
    // its pixels, so the recurrence is unchanged.  E rows start at zero (the
    // weights of skipped (Gaussian, pixel) pairs).
    const unsigned int qb0 = (unsigned int)__ballot(qmask & 1u), qb1 = (unsigned int)__ballot((qmask >> 1) & 1u);
    const unsigned int qb2 = (unsigned int)__ballot((qmask >> 2) & 1u), qb3 = (unsigned int)__ballot((qmask >> 3) & 1u);
    {
      float4* e4 = reinterpret_cast<float4*>(E);
      for (int c = lane; c < B * (kEStride / 4); c += 64) e4[c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    unsigned long long any_e = 0ull;           // pixels with some e > 0 in this batch
    __syncthreads();
    if (!all_done) {
      // One Gaussian, without branches.  T is -1 on a finished pixel (or one
      // outside the image) and at least kTMin otherwise, so a Gaussian below
      // the alpha threshold can run the same arithmetic with alpha = 0: testT
      // = T exactly, E = 0, T kept; on a finished pixel testT < 0 fails the
      // kTMin test and T stays -1.  Slot B is a Gaussian never taken (qmax < 0).
      auto step = [&](int k, const float4& c0, const float4& c1, float cq) {
        // c0 = (hx, hy, fx, fy), c1 = (l00, l10, l11, opacity), cq = qmax
        const float dx = (pcx - c0.x) - c0.z, dy = (pcy - c0.y) - c0.w;
        const float u = fmaf(c1.x, dx, c1.y * dy), v = c1.z * dy;
        const float q = fmaf(u, u, v * v);
        const bool take = q <= cq;             // alpha >= 1/255
        const float alpha = take ? fminf(kAlphaMax, c1.w * __builtin_amdgcn_exp2f(-q)) : 0.0f;
        const float testT = T * (1.0f - alpha);
        const bool keep = testT >= kTMin;
        const float e = keep ? alpha * T : 0.0f;   // > 0 exactly when the Gaussian was taken and kept
        if (k < B) E[k * kEStride + lane] = e;
        T = keep ? testT : -1.0f;
        const unsigned long long kb = __ballot(e > 0.0f);   // scalar bookkeeping
        any_e |= kb;
        count += (unsigned long long)__popcll(kb);
      };
      unsigned int bq = (qd & 2) ? ((qd & 1) ? qb3 : qb2) : ((qd & 1) ? qb1 : qb0);
      const int nsteps = max(max(__popc(qb0), __popc(qb1)), max(__popc(qb2), __popc(qb3)));
      auto next = [&]() {
        const int k = bq ? __ffs(bq) - 1 : B;
        bq &= bq - 1u;
        return k;
      };
      // two register sets alternate so that each step's splat is read from
      // LDS one step ahead without copies
      int ka = next();
      float4 a0 = s_bs[2 * ka], a1 = s_bs[2 * ka + 1];
      float aq = s_q[ka];
      for (int k = 0; k < nsteps; k += 2) {
        const int kb2 = next();
        const float4 b0v = s_bs[2 * kb2], b1v = s_bs[2 * kb2 + 1];
        const float bq2 = s_q[kb2];
        step(ka, a0, a1, aq);
        if (k + 1 >= nsteps) break;
        ka = next();
        a0 = s_bs[2 * ka]; a1 = s_bs[2 * ka + 1]; aq = s_q[ka];
        step(kb2, b0v, b1v, bq2);
        if (__ballot(T > 0.0f) == 0ull) break;
      }
    }
    // bit k: E row k belongs to this batch's Gaussian k (zero where it was not
    // evaluated); none when no pixel got a weight
    const unsigned long long contributed = any_e ? (nb >= 32 ? 0xFFFFFFFFull : (1ull << nb) - 1ull) : 0ull;
    __syncthreads();
    if (two_class) {
      // lane group g sums Gaussian gk's row over the group's pixels of each
      // class; stale rows are not read
      float S0 = 0.0f, S1 = 0.0f;
      if (gk < nb && ((contributed >> gk) & 1ull)) {
        const float4* row4 = reinterpret_cast<const float4*>(E + gk * kEStride + gq0);
        if (full0) {
#pragma unroll
          for (int q = 0; q < B / 4; ++q) {
            const float4 x = row4[q];
            S0 += (x.x + x.y) + (x.z + x.w);
          }
        } else {
          const unsigned int b0 = (unsigned int)(cm0 >> gq0), b1 = (unsigned int)(cm1 >> gq0);
#pragma unroll
          for (int q = 0; q < B / 4; ++q) {
            const float4 x = row4[q];
            const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              S0 += ((b0 >> (4 * q + m)) & 1u) ? xs[m] : 0.0f;
              S1 += ((b1 >> (4 * q + m)) & 1u) ? xs[m] : 0.0f;
            }
          }
        }
      }
#pragma unroll
      for (int o = B; o < 64; o <<= 1) {       // combine the lane groups
        S0 += __shfl_xor(S0, o, 64);
        S1 += __shfl_xor(S1, o, 64);
      }
      // the pair's record slots; binning cleared every pair's slots to (no
      // region, 0), which readers skip like any zero weight, so a pair whose
      // weights are both zero is not written
      if (lane < nb) {
        const unsigned int p = s_pidx[lane];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          if (l >= n_levels) break;
          const int c0 = (key0 >> (2 * l)) & 3, c1 = (key1 >> (2 * l)) & 3;
          const float w0 = (c0 == 0 ? S0 : 0.0f) + (c1 == 0 ? S1 : 0.0f);
          const float w1 = (c0 == 1 ? S0 : 0.0f) + (c1 == 1 ? S1 : 0.0f);
          if (w0 != 0.0f || w1 != 0.0f) {
            float2* rec = args.lv[l].records;
            rec[2ull * p] = make_float2(__int_as_float(rg0[l]), w0);
            rec[2ull * p + 1] = make_float2(__int_as_float(rg1[l]), w1);
          }
        }
      }
    } else {
    // W = E M on the matrix cores; stale E rows are replaced by zero below
    f4v acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    if (contributed) {
      const float* e0 = E + (lane & 15) * kEStride + 16 * kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float4 x = *reinterpret_cast<const float4*>(e0 + 16 * t * kEStride + 4 * q);
          const float xa[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const float bv = (float)((mbits >> (4 * q + m)) & 1u);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[m], bv, acc[t], 0, 0, 0);
          }
        }
      }
    }
    // lane holds W[g][col] for g = 16 t + 4 kk + r in acc[t][r]; stale rows count as zero
    auto wval = [&](int i) {
      const int g = 16 * (i >> 2) + 4 * kk + (i & 3);
      const float a = acc[i >> 2][i & 3];
      return ((contributed >> g) & 1ull) ? a : 0.0f;
    };
    if (rec_col) {                             // the pairs' record slots of nonzero weight (as above)
      const float rg = __int_as_float(col_greg);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const uint4 p4 = *reinterpret_cast<const uint4*>(&s_pidx[16 * t + 4 * kk]);
        const unsigned int pp[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (16 * t + 4 * kk + r < nb) {
            const float w = wval(4 * t + r);
            if (w != 0.0f) rec_out[2ull * pp[r] + (col & 1)] = make_float2(rg, w);
          }
      }
    }
    if (n_ext > 0) {                           // further-region columns: this batch's entry slots
      unsigned int ovf = 0u;
      if (ext_col) {
        const unsigned long long row0 = ebase + (unsigned long long)b0 * n_ext + (unsigned long long)(col - 2 * n_levels);
#pragma unroll
        for (int i = 0; i < 4 * NT; ++i) {
          const int g = 16 * (i >> 2) + 4 * kk + (i & 3);
          if (g < nb) {
            const unsigned long long slot = row0 + (unsigned long long)g * n_ext;
            const float w = wval(i);
            if (slot < args.extra_cap)
              args.extra[slot] = make_float4(__uint_as_float(s_gid[g]), __int_as_float(col_level),
                                             __int_as_float(col_greg), w);
            else if (w > 0.0f)
              ovf |= 1u << i;
          }
        }
      }
      if (__ballot(ovf != 0u)) {               // entry buffer full: add directly
        const int* ci = nullptr; const float* cv = nullptr; const float* dF = nullptr;
        float* ac = nullptr; float* zs = nullptr; int kc = 0, dd = 0;
#pragma unroll
        for (int l = 0; l < NL; ++l)
          if (l == col_level) {
            ci = args.lv[l].code_idx; cv = args.lv[l].code_val; kc = args.lv[l].k_code;
            dF = args.lv[l].dense_F; dd = args.lv[l].dense_d; ac = args.lv[l].acc; zs = args.lv[l].zsum;
          }
#pragma unroll
        for (int i = 0; i < 4 * NT; ++i)
          if ((ovf >> i) & 1u)
            add_region_direct(ci, cv, kc, dF, dd, ac, zs, s_gid[16 * (i >> 2) + 4 * kk + (i & 3)], col_greg,
                              wval(i), m_atoms, st);
      }
    }
    }
    if (spill && contributed) {  // regions without a column (many regions in the block): one at a time
      const bool had = gk < nb && ((contributed >> gk) & 1ull);
      const float* row = E + gk * kEStride + gq0;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        if (l >= n_levels || !((spill >> l) & 1u)) continue;
        const LevelView& lv = args.lv[l];
        const int reg = regs[l];
        unsigned long long rest = __ballot(reg >= 0) & ~s_excl[l];
        while (rest) {
          const int rr = __builtin_amdgcn_readlane(reg, __ffsll((long long)rest) - 1);
          const unsigned long long same = __ballot(reg == rr) & rest;
          rest &= ~same;
          // lane gk of each lane group sums Gaussian gk's weights over the region's pixels in the group
          float wr = 0.0f;
          if (had) {
            const unsigned long long mr = same >> gq0;
            for (int q = 0; q < B; ++q)
              if ((mr >> q) & 1ull) wr += row[q];
          }
#pragma unroll
          for (int o = B; o < 64; o <<= 1) wr += __shfl_xor(wr, o, 64);
          if (lane < nb && had && wr > 0.0f)
            add_region_direct(lv.code_idx, lv.code_val, lv.k_code, lv.dense_F, lv.dense_d, lv.acc, lv.zsum, my_id,
                              lv.region_base + rr, wr, m_atoms, st);
        }
      }
    }
    key_cur = key_next;
    key_next = key_after;
    sp_cur = sp_next;
    off_cur = off_next;
    __syncthreads();
  }
  if (lane == 0 && count) atomicAdd(&st->contrib, count);
}

// Eq. 6 on one row held by a wave (values in LDS or global memory).
template <int NS>
__device__ __forceinline__ void topk_row(const float* row, int m, int k, int lane, int* out_idx, float* out_val) {
  unsigned long long key[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int j = s * 64 + lane;
    const float v = j < m ? row[j] : 0.0f;
    key[s] = v > 0.0f ? (((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xffffffffu - (unsigned)j))
                      : 0ull;
  }
  int sel_i = -1;
  float sel_v = 0.0f, sum = 0.0f;
  for (int r = 0; r < k; ++r) {
    unsigned long long best = 0ull;
#pragma unroll
    for (int s = 0; s < NS; ++s) best = key[s] > best ? key[s] : best;
    best = wave_max_u64(best);
    if (best == 0ull) break;
    const unsigned int j = 0xffffffffu - (unsigned int)(best & 0xffffffffull);
    const float v = __uint_as_float((unsigned int)(best >> 32));
    sum += v;
    if (lane == r) { sel_i = (int)j; sel_v = v; }
    if ((int)(j & 63u) == lane) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == (int)(j >> 6)) key[s] = 0ull;
    }
  }
  if (lane < k) {
    out_idx[lane] = sel_i;
    out_val[lane] = sel_i >= 0 ? sel_v / sum : 0.0f;
  }
}

// Entropy of one row's distribution (App. C.2): H = -sum p log p with
// p = w / sum w over the strictly positive entries; 0 for an all-zero row.
__device__ __forceinline__ float row_entropy(const float* row, int m, int lane) {
  float s = 0.0f;
  for (int j = lane; j < m; j += 64) s += fmaxf(row[j], 0.0f);
  s = wave_sum(s);
  if (!(s > 0.0f)) return 0.0f;
  const float inv = 1.0f / s;
  float h = 0.0f;
  for (int j = lane; j < m; j += 64) {
    const float p = row[j] * inv;
    if (p > 0.0f) h -= p * logf(p);
  }
  return wave_sum(h);
}

// ---------------------------------------------------------------------------
// row build: G (a power of two <= 16) consecutive Gaussians per workgroup,
// their rows (stride M+1) in LDS; wave w walks views w, w+4, ...  The
// records of the G Gaussians in one view are one contiguous range
// (Gaussian-major), so the wave reads it 64 records at a time, coalesced; each
// lane finds its record's Gaussian by comparing against the G range starts
// (wave-uniform), runs of equal (Gaussian, region) records are folded, and
// each run adds its region's code with LDS atomic adds.  Rows are written
// back coalesced, Top-K and entropy read from LDS.  A wave's time goes to
// waiting on its chunk chain (loads, then cross-lane steps), so the register
// budget is set for more waves per SIMD: 64 VGPRs (eight waves) with two code
// quads, 96 (five) with four; the few spills fall outside the view loop.
// ---------------------------------------------------------------------------
template <int NS, int QN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QN <= 2 ? 8 : 5))) void k_rowbuild(RowBuildArgs a, int G) {
  extern __shared__ float rows[];            // G * (M+1)
  const int M = a.m_atoms, stride = M + 1;
  const long long i0 = (long long)blockIdx.x * G;
  const int gn = (int)min((long long)G, a.n - i0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  float* acc = a.acc + i0 * M;
  for (int g = wave; g < gn; g += 4)          // one row a wave, lanes along the row
    for (int j = lane; j < M; j += 64) rows[g * stride + j] = acc[(long long)g * M + j];
  __syncthreads();
  const unsigned int cap = (unsigned int)a.capacity;
  const bool vec = (a.k_code & 3) == 0 &&
                   ((reinterpret_cast<uintptr_t>(a.code_idx) | reinterpret_cast<uintptr_t>(a.code_val)) & 15) == 0;
  // first record of Gaussian `lane` (lanes 0..gn) in view v
  auto load_ob = [&](int v) -> unsigned int {
    if (v >= a.n_views || lane > gn) return 0u;
    return 2u * min(a.offsets[(long long)v * (a.n + 1) + i0 + lane], cap);
  };
  // record r of view v; past the view's range (or the views) the load still
  // goes to a record of the batch, so it is issued unconditionally, and the
  // value is dropped by the range test
  const unsigned int rec_last = 2u * cap - 1u;
  auto load_rec = [&](int v, unsigned int r) -> float2 {
    return a.records[(long long)max(0, min(v, a.n_views - 1)) * 2 * a.capacity + min(r, rec_last)];
  };
  // the view's record starts of Gaussians 1..G-1 as wave-uniform values (past
  // the group: never reached), so a record's Gaussian is a count of compares
  unsigned int sk[16];
  auto set_starts = [&](unsigned int ob) {
#pragma unroll
    for (int k = 1; k < 16; ++k)
      sk[k] = k < gn ? (unsigned int)__builtin_amdgcn_readlane((int)ob, k) : 0xFFFFFFFFu;
  };
  // Records of one 64-record chunk (record r of lane) folded per (Gaussian,
  // region): equal (Gaussian, region) records sit two lanes apart (the same
  // slot of consecutive pairs), so a segmented sum along lanes of equal
  // parity folds each run of them, and the run's last lane adds its code once
  // (fewer LDS atomics, which would otherwise collide on the same row
  // entries).  Returns whether this lane adds, with its row, region and weight.
  auto fold = [&](unsigned int r, unsigned int r1, float2 rc, int& g, int& reg, float& w) -> bool {
    g = 0;                                     // last Gaussian whose range starts at or before r
#pragma unroll
    for (int k = 1; k < 16; ++k) g += r >= sk[k] ? 1 : 0;
    reg = __float_as_int(rc.x);
    const bool valid = r < r1 && rc.y != 0.0f && reg >= 0 && reg < a.r_total;
    const int gk = valid ? g : -1;
    const int pg = __shfl_up(gk, 2, 64), pr = __shfl_up(reg, 2, 64);
    bool head = !valid || lane < 2 || pg != gk || pr != reg;
    // the lane ends its run when the record two lanes on starts a run (or is
    // past the chunk)
    const bool next_head = __shfl_down((int)head, 2, 64) != 0;
    w = valid ? rc.y : 0.0f;
    // one shuffle per step: a weight is positive (records hold sums of e > 0)
    // or, on an invalid lane, zero, so the run-head flag rides in the sign bit;
    // the steps stop once every lane's sum reaches back to its run's head
#pragma unroll
    for (int d = 2; d < 64; d <<= 1) {
      if (__ballot(!head) == 0ull) break;
      const float u = __shfl_up(head ? -w : w, d, 64);
      if (lane >= d && !head) { w += fabsf(u); head = __builtin_signbit(u) != 0; }
    }
    return valid && (lane >= 62 || next_head);
  };
  // branch-free: a slot outside [0, M) adds zero to the row's pad entry M
  // (never written back); an index >= M is flagged once per wave at the end
  bool code_err = false;
  auto add_code = [&](float* row, float w, int j, float c) {
    code_err |= j >= M;
    const bool ok = (unsigned int)j < (unsigned int)M;
    atomicAdd(&row[ok ? j : M], ok ? w * c : 0.0f);
  };
  // Codes of up to 4 QN slots in 16-byte rows (QN quads): a chunk's code
  // loads are issued (unconditionally, an inactive lane reading region 0,
  // quads past k_code re-reading the first) before the previous chunk's
  // adds, which use codes loaded one chunk earlier.
  const bool piped = a.k_code <= 4 * QN && a.r_total > 0 && (a.k_code & 3) == 0 &&
                     ((reinterpret_cast<uintptr_t>(a.code_idx) | reinterpret_cast<uintptr_t>(a.code_val)) & 15) == 0;
  const int nq = a.k_code >> 2;                // code quads per region (piped)
  bool p_act = false;
  int p_g = 0;
  float p_w = 0.0f;
  int4 p_j[QN];
  float4 p_c[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) { p_j[q] = make_int4(-1, -1, -1, -1); p_c[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f); }
  auto add_pending = [&]() {
    if (!p_act) return;
    float* row = rows + p_g * stride;
#pragma unroll
    for (int q = 0; q < QN; ++q)
      if (q < nq) {
        add_code(row, p_w, p_j[q].x, p_c[q].x); add_code(row, p_w, p_j[q].y, p_c[q].y);
        add_code(row, p_w, p_j[q].z, p_c[q].z); add_code(row, p_w, p_j[q].w, p_c[q].w);
      }
  };
  auto add_chunk = [&](unsigned int r, unsigned int r1, float2 rc) {
    int g, reg;
    float w;
    const bool act = fold(r, r1, rc, g, reg, w);
    if (piped) {
      const long long gr = (long long)(act ? reg : 0) * a.k_code;
      int4 j[QN];
      float4 c[QN];
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const long long gq = q < nq ? gr + 4 * q : gr;
        j[q] = *reinterpret_cast<const int4*>(a.code_idx + gq);
        c[q] = *reinterpret_cast<const float4*>(a.code_val + gq);
      }
      add_pending();
      p_act = act; p_g = g; p_w = w;
#pragma unroll
      for (int q = 0; q < QN; ++q) { p_j[q] = j[q]; p_c[q] = c[q]; }
      return;
    }
    if (!act) return;
    float* row = rows + g * stride;
    const long long gr = (long long)reg * a.k_code;
    for (int c = 0; c < a.k_code; c += 4) {   // four slots' loads before their adds
      int jj[4];
      float cv[4];
      if (vec) {
        const int4 ji = *reinterpret_cast<const int4*>(a.code_idx + gr + c);
        const float4 jv = *reinterpret_cast<const float4*>(a.code_val + gr + c);
        jj[0] = ji.x; jj[1] = ji.y; jj[2] = ji.z; jj[3] = ji.w;
        cv[0] = jv.x; cv[1] = jv.y; cv[2] = jv.z; cv[3] = jv.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          jj[u] = c + u < a.k_code ? a.code_idx[gr + c + u] : -1;
          cv[u] = c + u < a.k_code ? a.code_val[gr + c + u] : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) add_code(row, w, jj[u], cv[u]);
    }
  };
  // wave w walks views w, w+4, ...; the next view's offsets are loaded two
  // views ahead and its first 128 records (a group's records in a view
  // usually fill one or two chunks) one view ahead of their use
  int v = wave;
  unsigned int ob_c = load_ob(v), ob_n = load_ob(v + 4);
  unsigned int r0_c = (unsigned int)__builtin_amdgcn_readlane((int)ob_c, 0);
  unsigned int r1_c = (unsigned int)__builtin_amdgcn_readlane((int)ob_c, gn);
  float2 rc_c = load_rec(v, r0_c + (unsigned int)lane);
  float2 rc_c2 = load_rec(v, r0_c + 64u + (unsigned int)lane);
  for (; v < a.n_views; v += 4) {
    const unsigned int ob_nn = load_ob(v + 8);
    const unsigned int r0_n = (unsigned int)__builtin_amdgcn_readlane((int)ob_n, 0);
    const unsigned int r1_n = (unsigned int)__builtin_amdgcn_readlane((int)ob_n, gn);
    const float2 rc_n = load_rec(v + 4, r0_n + (unsigned int)lane);
    const float2 rc_n2 = load_rec(v + 4, r0_n + 64u + (unsigned int)lane);
    set_starts(ob_c);
    add_chunk(r0_c + (unsigned int)lane, r1_c, rc_c);
    if (r0_c + 64u < r1_c) add_chunk(r0_c + 64u + (unsigned int)lane, r1_c, rc_c2);
    for (unsigned int base = r0_c + 128u; base < r1_c; base += 64u) {
      const unsigned int r = base + (unsigned int)lane;
      add_chunk(r, r1_c, load_rec(v, r));
    }
    ob_c = ob_n; ob_n = ob_nn;
    r0_c = r0_n; r1_c = r1_n;
    rc_c = rc_n; rc_c2 = rc_n2;
  }
  add_pending();
  if (__ballot(code_err) != 0ull && lane == 0) atomicOr(&a.status->data_error, 2u);
  __syncthreads();
  for (int g = wave; g < gn; g += 4)
    for (int j = lane; j < M; j += 64) acc[(long long)g * M + j] = rows[g * stride + j];
  if (a.k_top > 0) {
    for (int g = wave; g < gn; g += 4)
      topk_row<NS>(rows + g * stride, M, a.k_top, lane, a.topk_idx + (i0 + g) * a.k_top,
                   a.topk_val + (i0 + g) * a.k_top);
  }
  if (a.entropy) {
    for (int g = wave; g < gn; g += 4) {
      const float h = row_entropy(rows + g * stride, M, lane);
      if (lane == 0) a.entropy[i0 + g] = h;
    }
  }
}

// ---------------------------------------------------------------------------
// Dense feature uplift (Eq. 3) on the same records: the decoded feature of
// every region, F_r = sum_slots c C[j] (Eq. 4), then one wave per Gaussian
// sums w F_r over its records (lanes split the D features) and divides by Z.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_region_features(const int* __restrict__ code_idx,
                                                         const float* __restrict__ code_val, long long r_total,
                                                         int k_code, const float* __restrict__ C, int m, int d,
                                                         float* __restrict__ F, Status* st) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= r_total * d) return;
  const long long r = t / d;
  const int c = (int)(t - r * d);
  float acc = 0.0f;
  for (int s = 0; s < k_code; ++s) {
    const int j = code_idx[r * k_code + s];
    if (j >= m) atomicOr(&st->data_error, 2u);
    else if (j >= 0) acc = fmaf(code_val[r * k_code + s], C[(long long)j * d + c], acc);
  }
  F[t] = acc;
}

__global__ __launch_bounds__(256) void k_rowbuild_dense(long long n, int d, const float* __restrict__ F,
                                                        long long r_total, int n_views,
                                                        const unsigned int* __restrict__ offsets,
                                                        const float2* __restrict__ records, long long capacity,
                                                        float* __restrict__ feat, float* __restrict__ zsum,
                                                        int accumulate, int final_pass) {
  const long long i = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  constexpr int kMaxPer = 16;                 // d <= 1024
  float acc[kMaxPer];
  const int per = (d + 63) / 64;
  float z = 0.0f;
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) acc[q] = 0.0f;
  if (accumulate) {   // running sums of earlier view batches (un-normalised)
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q)
      if (q < per && q * 64 + lane < d) acc[q] = feat[i * d + q * 64 + lane];
    z = zsum[i];
  }
  const unsigned int cap = (unsigned int)capacity;
  for (int v = 0; v < n_views; ++v) {
    const unsigned int* offv = offsets + (long long)v * (n + 1) + i;
    const unsigned int lo = min(offv[0], cap), hi = min(offv[1], cap);
    const float2* recv = records + (long long)v * 2 * capacity;
    for (unsigned int r = 2 * lo; r < 2 * hi; ++r) {
      const float2 rc = recv[r];
      const int reg = __float_as_int(rc.x);
      if (rc.y == 0.0f || reg < 0 || reg >= r_total) continue;
      z += rc.y;
      const float* fr = F + (long long)reg * d;
#pragma unroll
      for (int q = 0; q < kMaxPer; ++q)
        if (q < per && q * 64 + lane < d) acc[q] = fmaf(rc.y, fr[q * 64 + lane], acc[q]);
    }
  }
  const float sc = final_pass ? (z > 0.0f ? 1.0f / z : 0.0f) : 1.0f;
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q)
    if (q < per && q * 64 + lane < d) feat[i * d + q * 64 + lane] = acc[q] * sc;
  if (lane == 0 && zsum) zsum[i] = z;
}

hipError_t launch_region_features(const int* code_idx, const float* code_val, long long r_total, int k_code,
                                  const float* C, int m, int d, float* F, Status* st, hipStream_t s) {
  const long long tot = r_total * d;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_region_features, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, code_idx, code_val,
                     r_total, k_code, C, m, d, F, st);
  return hipGetLastError();
}

hipError_t launch_rowbuild_dense(long long n, int d, const float* F, long long r_total, int n_views,
                                 const unsigned int* offsets, const float2* records, long long capacity,
                                 float* feat, float* zsum, int accumulate, int final_pass, hipStream_t s) {
  if (n == 0) return hipSuccess;
  StageTimer::begin(kStRowBuild, s);
  hipLaunchKernelGGL(k_rowbuild_dense, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, d, F, r_total, n_views,
                     offsets, records, capacity, feat, zsum, accumulate, final_pass);
  StageTimer::end(kStRowBuild, s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_entropy(const float* __restrict__ acc, long long n, int m,
                                                 float* __restrict__ out) {
  const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const float h = row_entropy(acc + row * (long long)m, m, lane);
  if (lane == 0) out[row] = h;
}

hipError_t launch_entropy(const float* acc, long long n, int m, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_entropy, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, acc, n, m, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Top-K per row of an accumulator in memory (one wave per row), Eq. 6
// ---------------------------------------------------------------------------
template <int NS>
__global__ __launch_bounds__(256) void k_topk(const float* __restrict__ acc, long long n, int m, int k,
                                              int* __restrict__ out_idx, float* __restrict__ out_val) {
  const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  topk_row<NS>(acc + row * (long long)m, m, k, lane, out_idx + row * k, out_val + row * k);
}

__global__ void k_add_u64(unsigned long long* dst, const Status* st) { *dst += st->contrib; }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// The deferred further-region weights of one view: w times the region's code
// (or feature, for the dense uplift) added to the Gaussian's accumulator row.
// One thread per (entry, code slot) -- or (entry, feature column), plus one
// for Z, in the dense uplift -- so that each thread makes one atomic add.
__global__ __launch_bounds__(256) void k_apply_extra(UpliftViewArgs a, int m_atoms, int width, Status* st) {
  if (st->view_overflow) return;
  const unsigned long long n = min(st->n_extra, (unsigned long long)a.extra_cap) * (unsigned long long)width;
  for (unsigned long long t = blockIdx.x * 256ull + threadIdx.x; t < n; t += gridDim.x * 256ull) {
    const unsigned long long e = t / (unsigned int)width;
    const int c = (int)(t - e * (unsigned int)width);
    const float4 r = a.extra[e];
    if (!(r.w > 0.0f)) continue;             // reserved slot of a Gaussian without weight there
    const int l = __float_as_int(r.y);
    const unsigned int id = __float_as_uint(r.x);
    const long long greg = __float_as_int(r.z);
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k)
      if (k == l && k < a.n_levels) {
        const LevelView& lv = a.lv[k];
        if (lv.dense_F) {
          if (c < lv.dense_d)
            atomic_add_f32(&lv.acc[(unsigned long long)id * lv.dense_d + c], r.w * lv.dense_F[greg * lv.dense_d + c]);
          else if (c == lv.dense_d)
            atomic_add_f32(&lv.zsum[id], r.w);
        } else if (c < lv.k_code) {
          const int jj = lv.code_idx[greg * lv.k_code + c];
          if (jj >= m_atoms) atomicOr(&st->data_error, 2u);
          else if (jj >= 0)
            atomic_add_f32(&lv.acc[(unsigned long long)id * m_atoms + jj], r.w * lv.code_val[greg * lv.k_code + c]);
        }
      }
  }
}

// Statistics: U_v, the distinct (Gaussian, region) pairs of level 0 that
// received a weight in the view, from its records (Gaussian of a record by a
// binary search over the pair offsets) and its deferred entries, inserted
// into an open-addressing set of 64-bit keys (Gaussian << 32 | region; a
// mixing hash, linear probing, key + 1 so that 0 marks an empty slot).  New
// keys are counted once per wave.
__device__ __forceinline__ bool touch_insert(unsigned long long* table, unsigned long long cap,
                                             unsigned long long key, Status* st) {
  key += 1ull;
  unsigned long long h = key;                  // 64-bit finaliser: every key bit reaches every hash bit
  h ^= h >> 33; h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  h %= cap;
  for (int probe = 0; probe < 256; ++probe) {
    const unsigned long long prev = atomicCAS(&table[h], 0ull, key);
    if (prev == 0ull) return true;
    if (prev == key) return false;
    h = h + 1 == cap ? 0ull : h + 1;
  }
  atomicAdd(&st->touch_lost, 1ull);
  return false;
}

__global__ __launch_bounds__(256) void k_touch_clear(unsigned long long* table, unsigned long long cap,
                                                     const Status* st) {
  if (st->view_overflow) return;
  for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < cap; i += gridDim.x * 256ull) table[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_touch_count(const float2* __restrict__ rec,
                                                     const unsigned int* __restrict__ off, long long n,
                                                     const float4* __restrict__ extra, unsigned int extra_cap,
                                                     unsigned long long* table, unsigned long long cap, Status* st) {
  if (st->view_overflow || n <= 0) return;
  const unsigned long long nr = 2ull * st->total_pairs;
  const unsigned long long total = nr + min(st->n_extra, (unsigned long long)extra_cap);
  const int lane = threadIdx.x & 63;
  for (unsigned long long t0 = blockIdx.x * 256ull; t0 < total; t0 += gridDim.x * 256ull) {
    const unsigned long long t = t0 + threadIdx.x;
    bool fresh = false;
    if (t < nr) {
      const float2 r = rec[t];
      const int reg = __float_as_int(r.x);
      if (r.y != 0.0f && reg >= 0) {
        const unsigned int p = (unsigned int)(t >> 1);   // pair of the record
        long long lo = 0, hi = n - 1;                     // last Gaussian whose pairs start at or before p
        while (lo < hi) {
          const long long mid = (lo + hi + 1) >> 1;
          if (off[mid] <= p) lo = mid; else hi = mid - 1;
        }
        fresh = touch_insert(table, cap, ((unsigned long long)lo << 32) | (unsigned int)reg, st);
      }
    } else if (t < total) {
      const float4 e = extra[t - nr];
      if (e.w > 0.0f && __float_as_int(e.y) == 0)
        fresh = touch_insert(table, cap, ((unsigned long long)__float_as_uint(e.x) << 32) |
                                             (unsigned int)__float_as_int(e.z), st);
    }
    const unsigned long long m = __ballot(fresh);
    if (lane == 0 && m) atomicAdd(&st->touches, (unsigned long long)__popcll(m));
  }
}

hipError_t launch_uplift_view(UpliftViewArgs& a, hipStream_t s) {
  hipError_t e = launch_bin_view(a.bin, s);
  if (e != hipSuccess) return e;
  const BinArgs& b = a.bin;
  StageTimer::begin(kStComposite, s);
  if (a.n_levels == 1)
    hipLaunchKernelGGL((k_composite_blk<kCompositeBatch, kCompositeWaves, 1>), dim3(b.n_tiles), dim3(64), 0, s,
                       b.splats, b.tile_start, b.tile_order, b.keys[b.sorted], b.tiles_x, b.cam.width, b.cam.height,
                       a.n_levels, a.m_atoms, a, b.status);
  else
    hipLaunchKernelGGL((k_composite_blk<kCompositeBatch, kCompositeWaves, kMaxLevels>), dim3(b.n_tiles), dim3(64), 0,
                       s, b.splats, b.tile_start, b.tile_order, b.keys[b.sorted], b.tiles_x, b.cam.width,
                       b.cam.height, a.n_levels, a.m_atoms, a, b.status);
  StageTimer::end(kStComposite, s);
  if (a.extra_cap > 0) {
    StageTimer::begin(kStApplyExtra, s);
    int width = 1;                            // threads per entry: the widest level's code or feature row
    for (int l = 0; l < a.n_levels; ++l)
      width = std::max(width, a.lv[l].dense_F ? a.lv[l].dense_d + 1 : a.lv[l].k_code);
    hipLaunchKernelGGL(k_apply_extra, dim3(std::min(2048u, (a.extra_cap + 255) / 256)), dim3(256), 0, s, a,
                       a.m_atoms, width, b.status);
    StageTimer::end(kStApplyExtra, s);
  }
  if (a.count_touches && b.n > 0) {          // the view's sort buffers are free once it is composited
    unsigned long long* table = b.keys[b.sorted ^ 1];
    const unsigned long long cap = (unsigned long long)b.capacity;
    hipLaunchKernelGGL(k_touch_clear, dim3(1024), dim3(256), 0, s, table, cap, (const Status*)b.status);
    hipLaunchKernelGGL(k_touch_count, dim3(2048), dim3(256), 0, s, (const float2*)a.lv[0].records,
                       (const unsigned int*)b.offsets, b.n, (const float4*)a.extra, a.extra_cap, table, cap,
                       b.status);
  }
  return hipGetLastError();
}

// Gaussians per row-build workgroup: a power of two, at most 16 (rows of at
// most 64 KB of LDS, small enough for several workgroups per CU)
int rowbuild_group(int m) {
  int g = 16;
  while (g > 1 && g * (m + 1) > 16384) g >>= 1;
  return g;
}

// the instance for the Top-K width (NS 64-entry slices of a row) and the
// piped code quads (two up to 8 code slots, four up to 16)
template <int QN>
static void launch_rowbuild_ns(const RowBuildArgs& a, int G, int grid, size_t lds, int ns, hipStream_t s) {
  if (ns <= 1) hipLaunchKernelGGL((k_rowbuild<1, QN>), dim3(grid), dim3(256), lds, s, a, G);
  else if (ns <= 2) hipLaunchKernelGGL((k_rowbuild<2, QN>), dim3(grid), dim3(256), lds, s, a, G);
  else if (ns <= 4) hipLaunchKernelGGL((k_rowbuild<4, QN>), dim3(grid), dim3(256), lds, s, a, G);
  else if (ns <= 8) hipLaunchKernelGGL((k_rowbuild<8, QN>), dim3(grid), dim3(256), lds, s, a, G);
  else if (ns <= 16) hipLaunchKernelGGL((k_rowbuild<16, QN>), dim3(grid), dim3(256), lds, s, a, G);
  else if (ns <= 32) hipLaunchKernelGGL((k_rowbuild<32, QN>), dim3(grid), dim3(256), lds, s, a, G);
  else hipLaunchKernelGGL((k_rowbuild<64, QN>), dim3(grid), dim3(256), lds, s, a, G);
}

hipError_t launch_rowbuild(const RowBuildArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int G = rowbuild_group(a.m_atoms);
  const int grid = (int)((a.n + G - 1) / G);
  const size_t lds = sizeof(float) * (size_t)G * (a.m_atoms + 1);
  const int ns = (a.m_atoms + 63) / 64;
  StageTimer::begin(kStRowBuild, s);
  if (a.k_code > 8 && a.k_code <= 16) launch_rowbuild_ns<4>(a, G, grid, lds, ns, s);
  else launch_rowbuild_ns<2>(a, G, grid, lds, ns, s);
  StageTimer::end(kStRowBuild, s);
  return hipGetLastError();
}

hipError_t launch_topk(const float* acc, long long n, int m, int k, int* idx, float* val, hipStream_t s) {
  const int nb = (int)((n + 3) / 4);
  if (n == 0) return hipSuccess;
  const int ns = (m + 63) / 64;
  StageTimer::begin(kStTopk, s);
  if (ns <= 1) hipLaunchKernelGGL(k_topk<1>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  else if (ns <= 2) hipLaunchKernelGGL(k_topk<2>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  else if (ns <= 4) hipLaunchKernelGGL(k_topk<4>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  else if (ns <= 8) hipLaunchKernelGGL(k_topk<8>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  else if (ns <= 16) hipLaunchKernelGGL(k_topk<16>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  else if (ns <= 32) hipLaunchKernelGGL(k_topk<32>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  else hipLaunchKernelGGL(k_topk<64>, dim3(nb), dim3(256), 0, s, acc, n, m, k, idx, val);
  StageTimer::end(kStTopk, s);
  return hipGetLastError();
}

hipError_t launch_add_contrib(unsigned long long* dst, const Status* st, hipStream_t s) {
  hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(1), 0, s, dst, st);
  return hipGetLastError();
}

}  // namespace scoup
