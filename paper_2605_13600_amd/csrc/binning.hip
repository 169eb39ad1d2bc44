// Projection and tile binning shared by the uplift, the render and the
// backward (Sec. 3: the 3DGS tile rasterizer whose blending weights feed
// Eq. 1-2; Eq. 1's "ordered from front to back"):
//
//   k_project     one thread per Gaussian: FP64 EWA projection -> GSplat,
//                 number of overlapped tiles n_i
//   scan          device-wide exclusive scan of n_i -> Gaussian-major pair
//                 offsets off_i (also the record slots of the uplift)
//   k_bin_count / k_bin_colscan / k_tile_scan_order / k_bin_place
//                 pairs grouped by tile in one counting pass: key (float32
//                 depth bits << 32 | i) of pair (i, t) placed in t's list,
//                 tile t owns [tile_start[t], tile_start[t+1]); the tile
//                 order for the compositing (longest list first)
//   (larger images: k_emit + stable LSD radix sort by tile id + k_tile_ranges
//    + k_tile_order)
//   k_sort_lists_wave / k_sort_lists_wg / k_sort_blocks
//                 each block list sorted by (depth, id): one wave in registers
//                 up to 512 pairs, 2 or 4 waves up to 2048, one workgroup in
//                 LDS up to kSortCap
//   k_sort_big    lists longer than kSortCap sorted in global memory
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

constexpr int kCountThreads = 1024;
constexpr int kCountGroups = 256;          // workgroups of the counting pass (at least)
constexpr int kCountMaxTiles = 49152;      // 16-bit LDS counters: 96 KB
constexpr int kCountPlaceLdsTiles = 24576;  // placing pass: tile starts + bases in LDS up to here (96 KB more)
constexpr int kScanLdsTiles = 32768;        // block-length scan: lengths staged in LDS up to here (128 KB)

// the uplift's record arrays of the current view, per level (pairs whose
// block the Gaussian cannot reach are never composited: zero records)
struct CullRecords {
  float2* rec[4];
  int n;
};


// ---------------------------------------------------------------------------
// projection (one thread per Gaussian), FP64 arithmetic, FP32 storage
// ---------------------------------------------------------------------------
// Inputs of one Gaussian, loaded once (one memory latency per thread).
struct GaussIn {
  double mx, my, mz;
  float o, q[4], ls[3];
};

__device__ __forceinline__ GaussIn load_gauss(const float* __restrict__ means, const float* __restrict__ log_scales,
                                              const float* __restrict__ quats, const float* __restrict__ opacities,
                                              long long i) {
  GaussIn g;
  g.mx = means[3 * i + 0]; g.my = means[3 * i + 1]; g.mz = means[3 * i + 2];
  g.o = opacities[i];
#pragma unroll
  for (int k = 0; k < 4; ++k) g.q[k] = quats[4 * i + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) g.ls[k] = log_scales[3 * i + k];
  return g;
}

// The EWA splat of one Gaussian in one camera and the number of
// (1 << tile_shift)-pixel blocks its box covers (0 = invisible).  Every
// operation is a separately rounded IEEE double operation (no fused
// multiply-adds), so any kernel that calls this gets bit-identical boxes:
// the pair count checked before a resumed uplift is the one its views use.
__device__ __forceinline__ unsigned int project_splat(const GaussIn& gi, const CamDev& cam, int tile_shift,
                                                      GSplat& s) {
#pragma clang fp contract(off)
  s.ix = 0; s.iy = 0; s.fx = 0.f; s.fy = 0.f;
  s.l00 = 0.f; s.l10 = 0.f; s.l11 = 0.f; s.opacity = 0.f;
  s.bx0 = 1; s.bx1 = 0; s.by0 = 1; s.by1 = 0;   // empty box = invisible
  s.depth_bits = 0u; s.live = 0u;
  // camera point p = R mu + t summed left to right (the view depth and its
  // float32 sort key are reproducible exactly)
  const double mx = gi.mx, my = gi.my, mz = gi.mz;
  const double x = (double)cam.R[0] * mx + (double)cam.R[1] * my + (double)cam.R[2] * mz + (double)cam.t[0];
  const double y = (double)cam.R[3] * mx + (double)cam.R[4] * my + (double)cam.R[5] * mz + (double)cam.t[1];
  const double z = (double)cam.R[6] * mx + (double)cam.R[7] * my + (double)cam.R[8] * mz + (double)cam.t[2];
  const double o = gi.o;
  const double lo = log(255.0 * o);
  if (!(z > (double)cam.near_z) || !(lo >= 0.0)) return 0u;

  // 3D covariance Sigma = R diag(exp(2 s)) R^T from the normalised quaternion
  double qw = gi.q[0], qx = gi.q[1], qy = gi.q[2], qz = gi.q[3];
  const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const double Rq[3][3] = {
      {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
      {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
      {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
  const double s2[3] = {exp(2.0 * (double)gi.ls[0]), exp(2.0 * (double)gi.ls[1]), exp(2.0 * (double)gi.ls[2])};
  double S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      S[a][b] = Rq[a][0] * s2[0] * Rq[b][0] + Rq[a][1] * s2[1] * Rq[b][1] + Rq[a][2] * s2[2] * Rq[b][2];

  // EWA Jacobian at the clamped camera point
  const double fx = cam.fx, fy = cam.fy;
  const double limx = 1.3 * ((double)cam.width / (2.0 * fx));
  const double limy = 1.3 * ((double)cam.height / (2.0 * fy));
  const double tx = fmin(limx, fmax(-limx, x / z)) * z;
  const double ty = fmin(limy, fmax(-limy, y / z)) * z;
  const double j00 = fx / z, j02 = -fx * tx / (z * z);
  const double j11 = fy / z, j12 = -fy * ty / (z * z);
  double T0[3], T1[3];   // T = J W, W the camera rotation
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    T0[b] = j00 * (double)cam.R[0 * 3 + b] + j02 * (double)cam.R[2 * 3 + b];
    T1[b] = j11 * (double)cam.R[1 * 3 + b] + j12 * (double)cam.R[2 * 3 + b];
  }
  double U0[3], U1[3];   // T Sigma
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    U0[b] = T0[0] * S[0][b] + T0[1] * S[1][b] + T0[2] * S[2][b];
    U1[b] = T1[0] * S[0][b] + T1[1] * S[1][b] + T1[2] * S[2][b];
  }
  const double sxx = U0[0] * T0[0] + U0[1] * T0[1] + U0[2] * T0[2] + 0.3;
  const double sxy = U0[0] * T1[0] + U0[1] * T1[1] + U0[2] * T1[2];
  const double syy = U1[0] * T1[0] + U1[1] * T1[1] + U1[2] * T1[2] + 0.3;
  const double det = sxx * syy - sxy * sxy;
  const double mux = fx * x / z + (double)cam.cx;
  const double muy = fy * y / z + (double)cam.cy;
  if (!(det > 0.0) || !(fabs(mux) < 1073741824.0) || !(fabs(muy) < 1073741824.0)) return 0u;
  // conservative pixel box of {alpha >= 1/255}: |dx| <= sqrt(2 ln(255 o) Sxx)
  const double r2 = 2.0 * lo;
  const double hx = sqrt(r2 * sxx), hy = sqrt(r2 * syy);
  double x0 = ceil(mux - hx - 0.5) - 1.0, x1 = floor(mux + hx - 0.5) + 1.0;
  double y0 = ceil(muy - hy - 0.5) - 1.0, y1 = floor(muy + hy - 0.5) + 1.0;
  x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
  x1 = fmin(x1, (double)(cam.width - 1)); y1 = fmin(y1, (double)(cam.height - 1));
  if (!(x0 <= x1) || !(y0 <= y1)) return 0u;

  // scaled factor of the conic: q = (l00 dx + l10 dy)^2 + (l11 dy)^2 = log2(e)/2 d^T conic d
  const double ks = 0.84932180028801904272;   // sqrt(log2(e) / 2)
  const double l00 = sqrt(syy / det), l10 = -sxy / sqrt(det * syy), l11 = 1.0 / sqrt(syy);
  const double flx = floor(mux), fly = floor(muy);
  s.ix = (int)flx; s.iy = (int)fly;
  s.fx = (float)(mux - flx); s.fy = (float)(muy - fly);
  if (s.fx >= 1.0f) { s.fx = 0.0f; s.ix += 1; }
  if (s.fy >= 1.0f) { s.fy = 0.0f; s.iy += 1; }
  s.l00 = (float)(l00 * ks); s.l10 = (float)(l10 * ks); s.l11 = (float)(l11 * ks);
  s.opacity = (float)o;
  s.bx0 = (int16_t)x0; s.bx1 = (int16_t)x1; s.by0 = (int16_t)y0; s.by1 = (int16_t)y1;
  s.depth_bits = __float_as_uint((float)z);
  const int tx0 = s.bx0 >> tile_shift, tx1 = s.bx1 >> tile_shift;
  const int ty0 = s.by0 >> tile_shift, ty1 = s.by1 >> tile_shift;
  return (unsigned int)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
}

__global__ __launch_bounds__(256) void k_project(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ opacities, long long n,
    CamDev cam, int tile_shift, GSplat* __restrict__ out, unsigned int* __restrict__ n_tiles) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GaussIn gi = load_gauss(means, log_scales, quats, opacities, i);
  asm volatile("" ::"v"(gi.o), "v"(gi.q[0]), "v"(gi.q[1]), "v"(gi.q[2]), "v"(gi.q[3]), "v"(gi.ls[0]),
               "v"(gi.ls[1]), "v"(gi.ls[2]));   // keeps the loads ahead of the visibility test
  GSplat s;
  const unsigned int nt = project_splat(gi, cam, tile_shift, s);
  if (nt > 0u) {
    const int tx0 = s.bx0 >> tile_shift, tx1 = s.bx1 >> tile_shift;
    const int ty0 = s.by0 >> tile_shift, ty1 = s.by1 >> tile_shift;
    const BlockCull bc(s, tile_shift, cam.width, cam.height);
    unsigned int live = 0u;
    int r = 0;
    for (int ty = ty0; ty <= ty1 && r < 32; ++ty)
      for (int tx = tx0; tx <= tx1 && r < 32; ++tx, ++r)
        if (bc.live(tx, ty)) live |= 1u << r;
    s.live = live;
  }
  out[i] = s;
  n_tiles[i] = nt;
}

// Pairs (Gaussian, block) of up to kCountCams views in one pass over the
// Gaussians: totals[v] += sum_i (blocks of i's box in view v), the counts the
// views' own projections will give (same device function).  Per-view sums are
// wave-reduced, then gathered in LDS, then one atomic per (workgroup, view).
__global__ __launch_bounds__(256) void k_count_view_pairs(const float* __restrict__ means,
                                                          const float* __restrict__ log_scales,
                                                          const float* __restrict__ quats,
                                                          const float* __restrict__ opacities, long long n,
                                                          CamBatch cams, int tile_shift,
                                                          unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long s_tot[kCountCams];
  if (threadIdx.x < kCountCams) s_tot[threadIdx.x] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (long long i0 = (long long)blockIdx.x * 256; i0 < n; i0 += (long long)gridDim.x * 256) {
    const long long i = i0 + threadIdx.x;
    const bool ok = i < n;
    const GaussIn gi = load_gauss(means, log_scales, quats, opacities, ok ? i : 0);
    for (int v = 0; v < cams.n; ++v) {
      GSplat s;
      unsigned long long c = ok ? (unsigned long long)project_splat(gi, cams.c[v], tile_shift, s) : 0ull;
      for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
      if (lane == 0 && c) atomicAdd(&s_tot[v], c);
    }
  }
  __syncthreads();
  if (threadIdx.x < cams.n && s_tot[threadIdx.x]) atomicAdd(&totals[threadIdx.x], s_tot[threadIdx.x]);
}

hipError_t launch_count_view_pairs(const float* means, const float* log_scales, const float* quats,
                                   const float* opacities, long long n, const CamBatch& cams, int tile_shift,
                                   unsigned long long* totals, hipStream_t s) {
  if (n <= 0 || cams.n <= 0) return hipSuccess;
  const long long nb = std::min<long long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_count_view_pairs, dim3((unsigned)nb), dim3(256), 0, s, means, log_scales, quats, opacities,
                     n, cams, tile_shift, totals);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of n unsigned values, in place, in three kernels
// (block sums, scan of the sums, block-local scan + offset).  2048 per block.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256 * kScanItems;

__device__ __forceinline__ unsigned long long block_exclusive_scan_256(unsigned long long v,
                                                                        unsigned long long* sh,
                                                                        unsigned long long* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned long long a = tid >= o ? sh[tid - o] : 0ull;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  const unsigned long long incl = sh[tid];
  *total = sh[255];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const unsigned int* __restrict__ in, long long n,
                                                     unsigned long long* __restrict__ part) {
  __shared__ unsigned long long sh[256];
  const long long b0 = (long long)blockIdx.x * kScanBlock;
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = b0 + (long long)k * 256 + threadIdx.x;
    if (i < n) s += in[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// one workgroup: exclusive scan of the block sums, total pairs and capacity check
__global__ __launch_bounds__(1024) void k_scan_top(unsigned long long* __restrict__ part, int nb,
                                                   unsigned long long capacity, Status* st) {
  __shared__ unsigned long long sh[1024];
  const int tid = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b = tid * per, e = min(nb, b + per);
  unsigned long long s = 0;
  for (int i = b; i < e; ++i) s += part[i];
  sh[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned long long a = tid >= o ? sh[tid - o] : 0ull;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  unsigned long long run = sh[tid] - s;
  const unsigned long long total = sh[1023];
  for (int i = b; i < e; ++i) {
    const unsigned long long v = part[i];
    part[i] = run;
    run += v;
  }
  if (tid == 0 && st) {
    st->n_big = 0u;
    st->n_extra = 0ull;
    const bool over = total > capacity;
    st->total_pairs = over ? 0u : (unsigned int)total;
    st->view_overflow = over ? 1u : 0u;
    if (over) st->any_overflow = 1u;
    const unsigned int t32 = total > 0xffffffffull ? 0xffffffffu : (unsigned int)total;
    if (t32 > st->max_pairs) st->max_pairs = t32;
  }
}

__global__ __launch_bounds__(256) void k_scan_down(unsigned int* __restrict__ data, long long n,
                                                   const unsigned long long* __restrict__ part,
                                                   unsigned int* __restrict__ total_out) {
  __shared__ unsigned long long sh[256];
  const long long b0 = (long long)blockIdx.x * kScanBlock;
  // each thread owns kScanItems consecutive elements
  const long long i0 = b0 + (long long)threadIdx.x * kScanItems;
  unsigned int v[kScanItems];
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (i0 + k < n) ? data[i0 + k] : 0u;
    s += v[k];
  }
  unsigned long long tot;
  unsigned long long run = block_exclusive_scan_256(s, sh, &tot) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (i0 + k < n) data[i0 + k] = (unsigned int)run;
    run += v[k];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) *total_out = (unsigned int)run;
}

// ---------------------------------------------------------------------------
// Gaussian-major pair emission
// ---------------------------------------------------------------------------
// Blocks the Gaussian cannot reach get the tile id n_tiles, which sorts after
// every list and belongs to none.
__global__ __launch_bounds__(256) void k_emit(GSplat* splats, long long n, int tiles_x,
                                              int n_tiles, int tile_shift, int W, int H,
                                              const unsigned int* __restrict__ off,
                                              unsigned int* __restrict__ tile_ids,
                                              unsigned long long* __restrict__ keys, int keep_off,
                                              const Status* st) {
  if (st->view_overflow) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GSplat s = splats[i];
  if (s.bx0 > s.bx1) return;
  const unsigned long long key = ((unsigned long long)s.depth_bits << 32) | (unsigned long long)i;
  const int tx0 = s.bx0 >> tile_shift, tx1 = s.bx1 >> tile_shift;
  const int ty0 = s.by0 >> tile_shift, ty1 = s.by1 >> tile_shift;
  unsigned int p = off[i];
  const BlockCull bc(s, tile_shift, W, H);
  int r = 0;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx, ++p, ++r) {
      const bool live = pair_live(s, bc, r, tx, ty);
      tile_ids[p] = live ? (unsigned int)(ty * tiles_x + tx) : (unsigned int)n_tiles;
      keys[p] = key;
    }
  if (keep_off) splats[i].depth_bits = off[i];   // the depth is in the keys now
}

// Every pair's uplift record slots start as (no region, 0): coalesced over
// the view's pairs; the compositing overwrites those of reachable blocks.
__global__ __launch_bounds__(256) void k_clear_records(CullRecords cull, const Status* st) {
  if (st->view_overflow) return;
  const unsigned long long n = st->total_pairs;
  const float4 z = make_float4(__int_as_float(-1), 0.0f, __int_as_float(-1), 0.0f);
  for (int l = 0; l < cull.n; ++l) {
    float4* r = reinterpret_cast<float4*>(cull.rec[l]);
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += gridDim.x * 256ull) r[i] = z;
  }
}

// ---------------------------------------------------------------------------
// Grouping by tile with one counting pass (images up to kCountMaxTiles
// tiles).  Workgroup w owns a contiguous range of Gaussians and counts its
// pairs per tile in LDS (two 16-bit counters per word); a column scan over
// the workgroups and a scan over tiles give every (workgroup, tile) its base;
// the placing pass re-walks the Gaussians and drops each key at base + a
// local LDS ticket.  The order inside a (workgroup, tile) run follows the
// tickets; the per-block sort by (depth, id) that follows makes the result
// independent of it.
// ---------------------------------------------------------------------------
// Calls f(tx, ty) for every reachable block of Gaussian g's box: the first
// 32 blocks (row-major) from its reachability bits, set bits only (the row
// of a bit by a multiply-shift, exact for r < 32), then any further blocks
// with the culling test itself (boxes of more than 32 blocks are rare).
template <typename F>
__device__ __forceinline__ void for_each_live_block(const GSplat& g, int tile_shift, int W, int H, F&& f) {
  const int tx0 = g.bx0 >> tile_shift, tx1 = g.bx1 >> tile_shift;
  const int ty0 = g.by0 >> tile_shift, ty1 = g.by1 >> tile_shift;
  const int bw = tx1 - tx0 + 1, nb = bw * (ty1 - ty0 + 1);
  const unsigned int inv = (65535u + (unsigned int)bw) / (unsigned int)bw;   // ceil(2^16 / bw)
  unsigned int m = g.live & (nb >= 32 ? 0xFFFFFFFFu : ((1u << nb) - 1u));
  while (m) {
    const int r = __ffs(m) - 1;
    m &= m - 1u;
    const int ry = (int)(((unsigned int)r * inv) >> 16);
    f(tx0 + r - ry * bw, ty0 + ry);
  }
  if (nb > 32) {
    const BlockCull bc(g, tile_shift, W, H);
    for (int r = 32; r < nb; ++r) {
      const int ry = r / bw, tx = tx0 + r - ry * bw, ty = ty0 + ry;
      if (bc.live(tx, ty)) f(tx, ty);
    }
  }
}

__global__ __launch_bounds__(kCountThreads) void k_bin_count(const GSplat* __restrict__ splats, long long n,
                                                             int tiles_x, int n_tiles, int tile_shift, int W, int H,
                                                             long long per_wg, unsigned int* __restrict__ hist,
                                                             const Status* st) {
  extern __shared__ unsigned int h[];                // ceil(n_tiles / 2) words
  if (st->view_overflow) return;
  const int nw = (n_tiles + 1) >> 1;
  for (int j = threadIdx.x; j < nw; j += kCountThreads) h[j] = 0u;
  __syncthreads();
  const long long i0 = (long long)blockIdx.x * per_wg;
  const long long i1 = min(n, i0 + per_wg);
  long long i = i0 + threadIdx.x;
  GSplat g_next;                                     // the thread's next splat, loaded an iteration ahead
  if (i < i1) g_next = splats[i];
  for (; i < i1; i += kCountThreads) {
    const GSplat g = g_next;
    if (i + kCountThreads < i1) g_next = splats[i + kCountThreads];
    if (g.bx0 > g.bx1) continue;
    for_each_live_block(g, tile_shift, W, H, [&](int tx, int ty) {
      const int t = ty * tiles_x + tx;
      atomicAdd(&h[t >> 1], 1u << (16 * (t & 1)));
    });
  }
  __syncthreads();
  unsigned int* row = hist + (long long)blockIdx.x * n_tiles;
  for (int t = threadIdx.x; t < n_tiles; t += kCountThreads) row[t] = (h[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
}

// hist[w][t] <- sum of hist[w'][t] over w' < w; tile_len[t] <- sum over all w.
// A workgroup covers 256 / nseg consecutive tiles; thread (seg, tile) holds
// the 32 counts of workgroups 32 seg .. 32 seg + 31 of its tile in registers
// (one round of loads), the segments' totals meet in LDS.
constexpr int kColSeg = 32;                  // counting workgroups per segment
__host__ __device__ inline int colscan_tiles_per_wg(int n_wg) { return 256 / ((n_wg + kColSeg - 1) / kColSeg); }

__global__ __launch_bounds__(256) void k_bin_colscan(unsigned int* __restrict__ hist, int n_wg, int n_tiles,
                                                     unsigned int* __restrict__ tile_len, const Status* st) {
  __shared__ unsigned int part[256];
  const int nseg = (n_wg + kColSeg - 1) / kColSeg;   // <= 256 / 8
  const int tpb = 256 / nseg;
  const int tl = threadIdx.x % tpb, seg = threadIdx.x / tpb;
  const int t = blockIdx.x * tpb + tl;
  const bool act = seg < nseg && t < n_tiles;
  if (st->view_overflow) {                     // empty lists; the view is retried
    if (act && seg == 0) tile_len[t] = 0u;
    return;
  }
  const int w0 = seg * kColSeg;
  unsigned int v[kColSeg];
  unsigned int sum = 0u;
#pragma unroll
  for (int k = 0; k < kColSeg; ++k) {
    v[k] = act && w0 + k < n_wg ? hist[(long long)(w0 + k) * n_tiles + t] : 0u;
    sum += v[k];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  if (!act) return;
  unsigned int run = 0u;
  for (int q = 0; q < seg; ++q) run += part[q * tpb + tl];
#pragma unroll
  for (int k = 0; k < kColSeg; ++k) {
    if (w0 + k < n_wg) hist[(long long)(w0 + k) * n_tiles + t] = run;
    run += v[k];
  }
  if (seg == nseg - 1) tile_len[t] = run;
}

__global__ __launch_bounds__(kCountThreads) void k_bin_place(GSplat* splats, long long n,
                                                             int tiles_x, int n_tiles, int tile_shift, int W, int H,
                                                             long long per_wg, const unsigned int* __restrict__ hist,
                                                             const unsigned int* __restrict__ tile_start,
                                                             unsigned long long* __restrict__ keys,
                                                             const unsigned int* __restrict__ pair_off,
                                                             const Status* st) {
  extern __shared__ unsigned int h[];         // tickets: ceil(n_tiles / 2) words, then (images
  if (st->view_overflow) return;               // up to kCountPlaceLdsTiles blocks) start + base
  const int nw = (n_tiles + 1) >> 1;           // of every block: n_tiles words
  const bool staged = n_tiles <= kCountPlaceLdsTiles;
  unsigned int* sb = h + nw;
  const unsigned int* base = hist + (long long)blockIdx.x * n_tiles;
  for (int j = threadIdx.x; j < nw; j += kCountThreads) h[j] = 0u;
  if (staged)
    for (int t = threadIdx.x; t < n_tiles; t += kCountThreads) sb[t] = tile_start[t] + base[t];
  __syncthreads();
  const long long i0 = (long long)blockIdx.x * per_wg;
  const long long i1 = min(n, i0 + per_wg);
  long long i = i0 + threadIdx.x;
  // the thread's next splat and pair offset, loaded an iteration ahead (the
  // offset is written over the splat's depth before this iteration's key
  // stores, so waiting for it never waits for them)
  GSplat g_next;
  unsigned int off_next = 0u;
  if (i < i1) {
    g_next = splats[i];
    if (pair_off) off_next = pair_off[i];
  }
  for (; i < i1; i += kCountThreads) {
    const GSplat g = g_next;
    const unsigned int off = off_next;
    if (i + kCountThreads < i1) {
      g_next = splats[i + kCountThreads];
      if (pair_off) off_next = pair_off[i + kCountThreads];
    }
    if (g.bx0 > g.bx1) continue;
    if (pair_off) splats[i].depth_bits = off;        // the depth is in the keys now
    const unsigned long long key = ((unsigned long long)g.depth_bits << 32) | (unsigned long long)i;
    for_each_live_block(g, tile_shift, W, H, [&](int tx, int ty) {
      const int t = ty * tiles_x + tx;
      const unsigned int sh = 16 * (t & 1);
      const unsigned int ticket = (atomicAdd(&h[t >> 1], 1u << sh) >> sh) & 0xFFFFu;
      keys[(staged ? sb[t] : tile_start[t] + base[t]) + ticket] = key;
    });
  }
}




int count_groups(long long n) {
  const long long need = (n + 65534) / 65535;              // at most 65535 Gaussians per 16-bit counter
  return (int)std::max<long long>(kCountGroups, need);
}

bool count_binning_ok(long long n, int n_tiles) {
  return n_tiles <= kCountMaxTiles && count_groups(n) <= 4 * kCountGroups;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (tile id, key) pairs by tile id, 7-bit digits
// (larger images)
// ---------------------------------------------------------------------------
constexpr int kRadixBits = 7;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixItems = 16;                   // per thread
constexpr int kRadixBlock = 256 * kRadixItems;    // per workgroup

__global__ __launch_bounds__(256) void k_radix_hist(const unsigned int* __restrict__ tid_in, int shift,
                                                    int nblocks, unsigned int* __restrict__ hist,
                                                    const Status* st) {
  __shared__ unsigned int h[kRadixBins];
  if (st->view_overflow) return;
  const long long n = st->total_pairs;
  if (threadIdx.x < kRadixBins) h[threadIdx.x] = 0u;
  __syncthreads();
  const long long b0 = (long long)blockIdx.x * kRadixBlock;
#pragma unroll
  for (int k = 0; k < kRadixItems; ++k) {
    const long long i = b0 + (long long)k * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[(tid_in[i] >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kRadixBins) hist[(long long)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Rounds of 256 consecutive elements; inside a round the order is wave-major,
// lane-minor, so a stable rank is: running digit offset of the block + same-
// digit elements of earlier waves in the round + same-digit earlier lanes.
__global__ __launch_bounds__(256) void k_radix_scatter(const unsigned int* __restrict__ tid_in,
                                                       const unsigned long long* __restrict__ key_in, int shift,
                                                       int nblocks, const unsigned int* __restrict__ hist,
                                                       unsigned int* __restrict__ tid_out,
                                                       unsigned long long* __restrict__ key_out,
                                                       const Status* st) {
  __shared__ unsigned int run[kRadixBins];
  __shared__ unsigned int wcnt[4][kRadixBins];
  if (st->view_overflow) return;
  const long long n = st->total_pairs;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid < kRadixBins) run[tid] = hist[(long long)tid * nblocks + blockIdx.x];
  for (int j = tid; j < 4 * kRadixBins; j += 256) (&wcnt[0][0])[j] = 0u;
  __syncthreads();
  const long long b0 = (long long)blockIdx.x * kRadixBlock;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kRadixItems; ++r) {
    const long long i = b0 + (long long)r * 256 + tid;
    const bool valid = i < n;
    unsigned int t = 0;
    unsigned long long kv = 0;
    if (valid) { t = tid_in[i]; kv = key_in[i]; }
    const unsigned int d = (t >> shift) & (kRadixBins - 1);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const unsigned long long bb = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const unsigned int inwave = (unsigned int)__popcll(peers & lt);
    if (valid && inwave == 0) wcnt[wave][d] = (unsigned int)__popcll(peers);
    __syncthreads();
    if (valid) {
      unsigned int before = 0;
      for (int w = 0; w < wave; ++w) before += wcnt[w][d];
      const unsigned int pos = run[d] + before + inwave;
      tid_out[pos] = t;
      key_out[pos] = kv;
    }
    __syncthreads();
    if (tid < kRadixBins) {
      run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
      wcnt[0][tid] = 0u; wcnt[1][tid] = 0u; wcnt[2][tid] = 0u; wcnt[3][tid] = 0u;
    }
    __syncthreads();
  }
}

// tile_start[t] = first sorted pair with tile id >= t (t = 0..n_tiles); tiles
// longer than sort_cap are appended to big_tiles for k_sort_big
__global__ __launch_bounds__(256) void k_tile_ranges(const unsigned int* __restrict__ tile_ids, int n_tiles,
                                                     unsigned int* __restrict__ tile_start, int sort_cap,
                                                     unsigned int* __restrict__ big_tiles, Status* st) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_tiles) return;
  const unsigned int n = st->view_overflow ? 0u : st->total_pairs;
  auto lower = [&](unsigned int x) {
    unsigned int lo = 0, hi = n;
    while (lo < hi) {
      const unsigned int mid = (lo + hi) >> 1;
      if (tile_ids[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  const unsigned int a = lower((unsigned int)t);
  tile_start[t] = a;
  if (t < n_tiles) {
    const unsigned int b = lower((unsigned int)t + 1u);
    if (b - a > (unsigned int)sort_cap) big_tiles[atomicAdd(&st->n_big, 1u)] = (unsigned int)t;
  }
}

// Tiles whose list exceeds the consumer's LDS sort capacity are sorted in
// place in global memory, one workgroup per listed tile (rare; correctness
// path for dense tiles).  A small fixed grid walks the list.
__global__ __launch_bounds__(1024) void k_sort_big(unsigned long long* __restrict__ keys,
                                                   const unsigned int* __restrict__ tile_start,
                                                   const unsigned int* __restrict__ big_tiles, const Status* st) {
  if (st->view_overflow) return;
  const unsigned int nbig = st->n_big;
  const int tid = threadIdx.x;
  for (unsigned int q = blockIdx.x; q < nbig; q += gridDim.x) {
    const unsigned int tile = big_tiles[q];
    const unsigned int start = tile_start[tile];
    const long long L = (long long)tile_start[tile + 1] - start;
    unsigned long long* s = keys + start;
    long long n2 = 1;
    while (n2 < L) n2 <<= 1;
    for (long long k = 2; k <= n2; k <<= 1) {
      const long long hk = k >> 1;
      for (long long i = tid; i < (n2 >> 1); i += 1024) {
        const long long blk = i / hk, off = i - blk * hk;
        const long long a = blk * k + off, b = blk * k + k - 1 - off;
        if (b < L) cmp_swap(&s[a], &s[b]);
      }
      __syncthreads();
      for (long long j = k >> 2; j >= 1; j >>= 1) {
        for (long long i = tid; i < (n2 >> 1); i += 1024) {
          const long long blk = i / j, off = i - blk * j;
          const long long a = blk * 2 * j + off, b = a + j;
          if (b < L) cmp_swap(&s[a], &s[b]);
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// Compositing order: tiles by list length, longest first, in buckets of one
// length each below kOrderBuckets - 1 and one bucket for all longer lists.
constexpr int kOrderBuckets = 2048;

// Depth order inside every block list: one workgroup of NT threads per block
// whose list has hi/2 < L <= hi = NT x PER pairs (one launch per size class),
// a bitonic network over hi keys (the list padded with ~0).  Thread t keeps
// elements t PER .. t PER + PER - 1 in registers: compare-exchange distances
// below PER stay in registers; longer ones go through LDS, stored element-
// slot-major (slot r of thread t at r NT + t) so that a wave's accesses are
// consecutive.
template <int PER, int J>
__device__ __forceinline__ void bitonic_regs(unsigned long long (&v)[PER], int base, int k) {
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if ((r & J) == 0) {
      const unsigned long long a = v[r], b = v[r ^ J];
      const bool asc = ((base + r) & k) == 0;
      const bool sw = asc ? (a > b) : (a < b);
      v[r] = sw ? b : a;
      v[r ^ J] = sw ? a : b;
    }
  }
}

template <int NT, int PER>
__device__ void sort_block_list(unsigned long long* __restrict__ s, int L, unsigned long long* sk) {
  constexpr int HI = NT * PER;
  const int t = threadIdx.x, base = t * PER;
  unsigned long long v[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) v[r] = base + r < L ? s[base + r] : ~0ull;
  for (int k = 2; k <= HI; k <<= 1) {
    for (int j = k >> 1; j >= PER; j >>= 1) {      // partner in thread t ^ (j / PER), same slot
#pragma unroll
      for (int r = 0; r < PER; ++r) sk[r * NT + t] = v[r];
      __syncthreads();
      const int pt = t ^ (j / PER);
      const bool lower = (base & j) == 0;
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const unsigned long long w = sk[r * NT + pt];
        const bool asc = ((base + r) & k) == 0;
        v[r] = (asc == lower) ? (v[r] < w ? v[r] : w) : (v[r] > w ? v[r] : w);
      }
      __syncthreads();
    }
    if (PER >= 8 && k >= 8) bitonic_regs<PER, (PER >= 8 ? 4 : 1)>(v, base, k);
    if (PER >= 4 && k >= 4) bitonic_regs<PER, (PER >= 4 ? 2 : 1)>(v, base, k);
    if (PER >= 2) bitonic_regs<PER, 1>(v, base, k);
  }
#pragma unroll
  for (int r = 0; r < PER; ++r)
    if (base + r < L) s[base + r] = v[r];
  __syncthreads();                             // sk is reused by the next list
}


template <int NT, int PER>
__global__ __launch_bounds__(NT) void k_sort_blocks(unsigned long long* __restrict__ keys,
                                                    const unsigned int* __restrict__ tile_start,
                                                    const unsigned int* __restrict__ order, int n_tiles, int lo,
                                                    const Status* st) {
  constexpr int HI = NT * PER;
  __shared__ unsigned long long sk[HI];
  if (st->view_overflow) return;
  // the order puts every list of at least kOrderBuckets - 1 keys first (the
  // only ones this size class can hold), so a workgroup stops at the first
  // shorter one
  for (int q = blockIdx.x; q < n_tiles; q += gridDim.x) {
    const int tile = (int)order[q];
    const unsigned int start = tile_start[tile];
    const int L = (int)(tile_start[tile + 1] - start);
    if (L < kOrderBuckets - 1) break;
    if (L <= lo || L > HI) continue;
    sort_block_list<NT, PER>(keys + start, L, sk);
  }
}


int radix_passes(int n_tiles) {
  int bits = 1;
  while ((1 << bits) < n_tiles) ++bits;
  return (bits + kRadixBits - 1) / kRadixBits;
}

long long radix_blocks(long long capacity) { return (capacity + kRadixBlock - 1) / kRadixBlock; }
long long scan_blocks(long long n) { return (n + kScanBlock - 1) / kScanBlock; }

// Processing order of the tiles for the compositing kernels: longest list
// first (lists of 2047 or more pairs share the first bucket), so that the
// blocks with the longest sequential loops start at the beginning of the
// launch instead of setting its tail.  One workgroup; a counting sort on the
// clamped length.

constexpr int kOrderLdsTiles = 32768;          // bucket of each tile kept in LDS up to this many tiles

__global__ __launch_bounds__(1024) void k_tile_order(const unsigned int* __restrict__ tile_start, int n_tiles,
                                                     unsigned int* __restrict__ order, const Status* st) {
  __shared__ unsigned int h[kOrderBuckets];
  __shared__ unsigned int part[1024];
  extern __shared__ unsigned short s_b[];      // [n_tiles] when n_tiles <= kOrderLdsTiles
  const int tid = threadIdx.x;
  if (st->view_overflow) {
    for (int t = tid; t < n_tiles; t += 1024) order[t] = (unsigned int)t;
    return;
  }
  for (int b = tid; b < kOrderBuckets; b += 1024) h[b] = 0u;
  __syncthreads();
  auto bucket = [&](int t) {
    const unsigned int L = tile_start[t + 1] - tile_start[t];
    return kOrderBuckets - 1 - (int)min(L, (unsigned int)(kOrderBuckets - 1));
  };
  const bool keep = n_tiles <= kOrderLdsTiles;
  for (int t = tid; t < n_tiles; t += 1024) {
    const int b = bucket(t);
    if (keep) s_b[t] = (unsigned short)b;
    atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  // exclusive scan of the buckets: two per thread, then across threads
  const unsigned int c0 = h[2 * tid], c1 = h[2 * tid + 1];
  part[tid] = c0 + c1;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned int v = tid >= o ? part[tid - o] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const unsigned int before = part[tid] - (c0 + c1);
  __syncthreads();
  h[2 * tid] = before;
  h[2 * tid + 1] = before + c0;
  __syncthreads();
  for (int t = tid; t < n_tiles; t += 1024) order[atomicAdd(&h[keep ? (int)s_b[t] : bucket(t)], 1u)] = (unsigned int)t;
}

// ---------------------------------------------------------------------------
// Depth order of a block list of at most 64 R keys by one wave: element
// e = r 64 + lane sits in register r of lane `lane`.  The bitonic network is
// the all-ascending form (per merge size k a mirror stage pairing e with
// e ^ (k - 1), then half-cleaners pairing e with e ^ j, the smaller key
// always to the lower index), so the ~0 padding past the list never moves
// down: registers holding padding only are skipped, and the network stops
// at the list's power-of-two size.  Distances of 64 and more pair registers
// of one lane; shorter ones exchange across lanes (DPP, swizzle or
// bpermute).  No LDS, no barriers.
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ int lane_xor(int v) {
  if constexpr (M == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  else if constexpr (M == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  else if constexpr (M == 3) return __builtin_amdgcn_update_dpp(0, v, 0x1B, 0xF, 0xF, false);   // quad_perm 3,2,1,0
  else if constexpr (M == 7) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  else if constexpr (M == 15) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false); // row_mirror
  else if constexpr (M < 32) return __builtin_amdgcn_ds_swizzle(v, (M << 10) | 0x1F);          // xor within 32
  else return __shfl_xor(v, M, 64);
}

template <int M>
__device__ __forceinline__ unsigned long long lane_xor64(unsigned long long x) {
  const unsigned int lo = (unsigned int)lane_xor<M>((int)(unsigned int)x);
  const unsigned int hi = (unsigned int)lane_xor<M>((int)(unsigned int)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// one cross-lane stage with partner lane ^ M; the lower index keeps the
// smaller key (`hb` = the partner's distinguishing lane bit)
template <int R, int M, int HB>
__device__ __forceinline__ void wave_cross_stage(unsigned long long (&v)[R], int rr, int lane) {
  const bool lower = (lane & HB) == 0;
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    if (r < rr) {
      const unsigned long long w = lane_xor64<M>(v[r]);
      const bool take = lower ? (w < v[r]) : (w > v[r]);
      v[r] = take ? w : v[r];
    }
  }
}

// half-cleaners j = jmax .. 1 for j < 64
template <int R>
__device__ __forceinline__ void wave_cross_cleaners(unsigned long long (&v)[R], int jmax, int rr, int lane) {
  if (jmax >= 32) wave_cross_stage<R, 32, 32>(v, rr, lane);
  if (jmax >= 16) wave_cross_stage<R, 16, 16>(v, rr, lane);
  if (jmax >= 8) wave_cross_stage<R, 8, 8>(v, rr, lane);
  if (jmax >= 4) wave_cross_stage<R, 4, 4>(v, rr, lane);
  if (jmax >= 2) wave_cross_stage<R, 2, 2>(v, rr, lane);
  if (jmax >= 1) wave_cross_stage<R, 1, 1>(v, rr, lane);
}

// register half-cleaner: registers r and r ^ S (S = j / 64)
template <int R, int S>
__device__ __forceinline__ void wave_reg_stage(unsigned long long (&v)[R], int rr) {
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    if ((r & S) || (r ^ S) >= rr) continue;
    const unsigned long long a = v[r], b = v[r ^ S];
    const bool sw = b < a;
    v[r] = sw ? b : a;
    v[r ^ S] = sw ? a : b;
  }
}

// mirror stage for k >= 128 (S = k / 64 - 1): register r pairs with register
// r ^ S of lane 63 - lane
template <int R, int S>
__device__ __forceinline__ void wave_mirror_stage(unsigned long long (&v)[R], int rr) {
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    if ((r ^ S) < r || (r ^ S) >= rr) continue;      // r is the lower register of the pair
    const unsigned long long a = v[r], b = v[r ^ S];
    const unsigned long long bm = lane_xor64<63>(b), am = lane_xor64<63>(a);
    v[r] = bm < a ? bm : a;
    v[r ^ S] = am > b ? am : b;
  }
}

// the network up to merge size n2 (<= 64 R) on one wave's registers
template <int R>
__device__ __forceinline__ void wave_sort_regs(unsigned long long (&v)[R], int n2, int rr, int lane) {
  for (int k = 2; k <= n2; k <<= 1) {
    if (k <= 64) {                             // mirror within k lanes
      switch (k) {
        case 2: wave_cross_stage<R, 1, 1>(v, rr, lane); break;
        case 4: wave_cross_stage<R, 3, 2>(v, rr, lane); break;
        case 8: wave_cross_stage<R, 7, 4>(v, rr, lane); break;
        case 16: wave_cross_stage<R, 15, 8>(v, rr, lane); break;
        case 32: wave_cross_stage<R, 31, 16>(v, rr, lane); break;
        default: wave_cross_stage<R, 63, 32>(v, rr, lane); break;
      }
    } else {                                   // mirror across registers, then register half-cleaners
      const int S = (k >> 6) - 1;
      if constexpr (R >= 2) if (S == 1) wave_mirror_stage<R, 1>(v, rr);
      if constexpr (R >= 4) if (S == 3) wave_mirror_stage<R, 3>(v, rr);
      if constexpr (R >= 8) if (S == 7) wave_mirror_stage<R, 7>(v, rr);
      const int jr = k >> 8;
      if constexpr (R >= 8) if (jr >= 4) wave_reg_stage<R, 4>(v, rr);
      if constexpr (R >= 4) if (jr >= 2) wave_reg_stage<R, 2>(v, rr);
      if constexpr (R >= 2) if (jr >= 1) wave_reg_stage<R, 1>(v, rr);
    }
    wave_cross_cleaners<R>(v, k <= 64 ? (k >> 2) : 32, rr, lane);
  }
}

template <int R>
__device__ __forceinline__ void wave_sort_list(unsigned long long* __restrict__ s, int L, int lane) {
  unsigned long long v[R];
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    const int e = r * 64 + lane;
    v[r] = e < L ? s[e] : ~0ull;
  }
  int n2 = 2;
  while (n2 < L) n2 <<= 1;
  wave_sort_regs<R>(v, n2, (L + 63) >> 6, lane);
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    const int e = r * 64 + lane;
    if (e < L) s[e] = v[r];
  }
}

constexpr int kWaveSortMax = 512;              // lists up to this length: one wave each
constexpr int kWgSortMax = 2048;               // up to this length: 2 or 4 waves of 512

// one wave per block list (longest first); lists of 2 .. kWaveSortMax keys
__global__ __launch_bounds__(256) void k_sort_lists_wave(unsigned long long* __restrict__ keys,
                                                         const unsigned int* __restrict__ tile_start,
                                                         const unsigned int* __restrict__ order, int n_tiles,
                                                         const Status* st) {
  if (st->view_overflow) return;
  const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (w >= n_tiles) return;
  const int lane = threadIdx.x & 63;
  const int tile = order ? (int)order[w] : w;
  const unsigned int start = tile_start[tile];
  const int L = (int)(tile_start[tile + 1] - start);
  if (L < 2 || L > kWaveSortMax) return;
  unsigned long long* s = keys + start;
  if (L <= 128) wave_sort_list<2>(s, L, lane);
  else if (L <= 256) wave_sort_list<4>(s, L, lane);
  else wave_sort_list<8>(s, L, lane);
}

// W waves per list of lo < L <= 512 W keys: each wave sorts its 512-key
// chunk in registers, then the merges of size 1024 .. 512 W pair waves
// through LDS (mirror and half-cleaners of 512 and more), registers
// (256 .. 64) and lanes (32 .. 1).
template <int W>
__device__ void wg_sort_list(unsigned long long* __restrict__ s, int L, unsigned long long* sx) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned long long v[8];
#pragma clang loop unroll(full)
  for (int r = 0; r < 8; ++r) {
    const int e = wave * 512 + r * 64 + lane;
    v[r] = e < L ? s[e] : ~0ull;
  }
  const int rr = min(8, max(0, (L - wave * 512 + 63) >> 6));
  wave_sort_regs<8>(v, 512, rr, lane);
  for (int k = 1024; k <= 512 * W; k <<= 1) {
    for (int j = k >> 1; j >= 512; j >>= 1) {  // j = k/2: mirror (partner e ^ (k - 1)); else e ^ j
      const bool mirror = j == (k >> 1);
      const int pw = mirror ? (wave ^ ((k >> 9) - 1)) : (wave ^ (j >> 9));
      const bool lower = wave < pw;
#pragma clang loop unroll(full)
      for (int r = 0; r < 8; ++r) sx[wave * 512 + r * 64 + lane] = v[r];
      __syncthreads();
#pragma clang loop unroll(full)
      for (int r = 0; r < 8; ++r) {
        const unsigned long long w = mirror ? sx[pw * 512 + (r ^ 7) * 64 + (lane ^ 63)] : sx[pw * 512 + r * 64 + lane];
        const bool take = lower ? (w < v[r]) : (w > v[r]);
        v[r] = take ? w : v[r];
      }
      __syncthreads();
    }
    wave_reg_stage<8, 4>(v, 8);
    wave_reg_stage<8, 2>(v, 8);
    wave_reg_stage<8, 1>(v, 8);
    wave_cross_cleaners<8>(v, 32, 8, lane);
  }
#pragma clang loop unroll(full)
  for (int r = 0; r < 8; ++r) {
    const int e = wave * 512 + r * 64 + lane;
    if (e < L) s[e] = v[r];
  }
}

// A bounded grid walks the compositing order (longest lists first) and stops
// at the first list of lo keys or fewer: no workgroup per block of the image.
template <int W>
__global__ __launch_bounds__(64 * W) void k_sort_lists_wg(unsigned long long* __restrict__ keys,
                                                          const unsigned int* __restrict__ tile_start,
                                                          const unsigned int* __restrict__ order, int n_tiles,
                                                          int lo, const Status* st) {
  __shared__ unsigned long long sx[W * 512];
  if (st->view_overflow) return;
  for (int q = blockIdx.x; q < n_tiles; q += gridDim.x) {
    const int tile = (int)order[q];
    const unsigned int start = tile_start[tile];
    const int L = (int)(tile_start[tile + 1] - start);
    if (L <= lo) break;
    if (L > 512 * W) continue;
    wg_sort_list<W>(keys + start, L, sx);
    __syncthreads();                           // sx is reused by the next list
  }
}

// Counting path, one workgroup: exclusive scan of the block list lengths
// (tile_start holds the lengths on entry, the starts on exit), the lists
// longer than sort_cap (big_tiles), and the compositing order, longest list
// first (as k_tile_order).  Thread i owns tiles [i c, i c + c) and loads
// their lengths into registers at once (C >= c, a compile-time bound, so the
// loads issue together instead of one latency per tile); after the scan of
// the 1024 chunk sums it rewrites them as starts and buckets them by length.
// Exclusive scan of one value per thread over a 1024-thread workgroup:
// shuffle scans inside the waves, then each thread adds the totals of the
// waves before it (16 wave totals in LDS; two barriers).
__device__ __forceinline__ unsigned int block_exclusive_scan_1024(unsigned int x, unsigned int* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned int inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned int v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  unsigned int before = 0u;
  for (int k = 0; k < w; ++k) before += wsum[k];
  __syncthreads();                             // wsum free for the next scan
  return before + inc - x;
}

template <int C>
__global__ __launch_bounds__(1024) void k_tile_scan_order(unsigned int* __restrict__ tile_start, int n_tiles,
                                                          int sort_cap, unsigned int* __restrict__ big_tiles,
                                                          unsigned int* __restrict__ order, Status* st) {
  __shared__ unsigned int h[kOrderBuckets];
  __shared__ unsigned int wsum[16];
  extern __shared__ unsigned int s_len[];      // staged: the lengths, then the starts (n_tiles words)
  const int tid = threadIdx.x;
  for (int b = tid; b < kOrderBuckets; b += 1024) h[b] = 0u;
  const bool overflow = st->view_overflow != 0;
  constexpr bool staged = 1024 * C <= kScanLdsTiles;   // every size this instance takes fits
  const int c = (n_tiles + 1023) / 1024;        // <= C
  const int t0 = min(n_tiles, tid * c), t1 = min(n_tiles, t0 + c);
  unsigned int len[C];
  if constexpr (staged) {
    // coalesced: thread i moves words i, i + 1024, ... (C loads in flight),
    // then reads its own chunk from LDS
#pragma unroll
    for (int k = 0; k < C; ++k) len[k] = tile_start[min(tid + 1024 * k, n_tiles - 1)];
#pragma unroll
    for (int k = 0; k < C; ++k)
      if (tid + 1024 * k < n_tiles) s_len[tid + 1024 * k] = len[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C; ++k) len[k] = t0 + k < t1 ? s_len[t0 + k] : 0u;
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) {              // unconditional (clamped) loads, then the range test
      const unsigned int x = tile_start[min(t0 + k, n_tiles - 1)];
      len[k] = t0 + k < t1 ? x : 0u;
    }
  }
  unsigned int sum = 0u;
#pragma unroll
  for (int k = 0; k < C; ++k) sum += len[k];
  unsigned int run = block_exclusive_scan_1024(sum, wsum);   // (the bucket clears above are before its barriers)
  if (tid == 1023) tile_start[n_tiles] = run + sum;
  auto bucket = [](unsigned int L) { return kOrderBuckets - 1 - (int)min(L, (unsigned int)(kOrderBuckets - 1)); };
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const int t = t0 + k;
    if (t < t1) {
      const unsigned int L = len[k];
      if (staged) s_len[t] = run; else tile_start[t] = run;
      run += L;
      atomicAdd(&h[bucket(L)], 1u);
      if (L > (unsigned int)sort_cap && !overflow) big_tiles[atomicAdd(&st->n_big, 1u)] = (unsigned int)t;
    }
  }
  __syncthreads();
  if (staged)                                   // the starts out, coalesced
    for (int j = tid; j < n_tiles; j += 1024) tile_start[j] = s_len[j];
  if (!order) return;
  // exclusive scan of the buckets: two per thread, then across threads
  const unsigned int c0 = h[2 * tid], c1 = h[2 * tid + 1];
  const unsigned int before = block_exclusive_scan_1024(c0 + c1, wsum);
  h[2 * tid] = before;
  h[2 * tid + 1] = before + c0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const int t = t0 + k;
    if (t < t1) order[atomicAdd(&h[bucket(len[k])], 1u)] = (unsigned int)t;
  }
}

// the per-thread tile bound of k_tile_scan_order
static void launch_tile_scan_order(const BinArgs& a, hipStream_t s) {
  const int c = (a.n_tiles + 1023) / 1024;
  const size_t lds = c <= kScanLdsTiles / 1024 ? sizeof(unsigned int) * (size_t)a.n_tiles : 0;
#define TSO(C)                                                                                                  \
  hipLaunchKernelGGL(k_tile_scan_order<C>, dim3(1), dim3(1024), lds, s, a.tile_start, a.n_tiles, a.sort_cap,    \
                     a.big_tiles, a.tile_order, a.status)
  if (c <= 16) TSO(16);
  else if (c <= 32) TSO(32);
  else TSO(kCountMaxTiles / 1024);
#undef TSO
}

hipError_t binning_set_lds_limits() {
  const int bytes = (int)sizeof(unsigned int) * (kCountMaxTiles / 2);
  hipError_t e = hipFuncSetAttribute((const void*)k_bin_count, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  // placing pass: 2 B of tickets + 4 B of start per block while staged (6 x 24576 B), else tickets only
  e = hipFuncSetAttribute((const void*)k_bin_place, hipFuncAttributeMaxDynamicSharedMemorySize,
                          std::max(bytes, 6 * kCountPlaceLdsTiles));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_tile_order, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sizeof(unsigned short) * kOrderLdsTiles);
  if (e != hipSuccess) return e;
  const int scan_lds = (int)sizeof(unsigned int) * kScanLdsTiles;
  if ((e = hipFuncSetAttribute((const void*)k_tile_scan_order<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               scan_lds)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_tile_scan_order<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               scan_lds)) != hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)k_tile_scan_order<kCountMaxTiles / 1024>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, scan_lds);
}

static CullRecords cull_of(const BinArgs& a) {
  CullRecords c{};
  c.n = std::min(a.n_cull_records, 4);
  for (int l = 0; l < c.n; ++l) c.rec[l] = a.cull_records[l];
  return c;
}

// depth order inside every tile list of the sorted buffer
static void sort_lists(const BinArgs& a, hipStream_t s, bool order_done) {
  if (a.tile_order && a.n_tiles > 0 && !order_done)
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), a.n_tiles <= kOrderLdsTiles ? 2 * (size_t)a.n_tiles : 0, s,
                       a.tile_start, a.n_tiles, a.tile_order, a.status);
  hipLaunchKernelGGL(k_sort_big, dim3(16), dim3(1024), 0, s, a.keys[a.sorted], a.tile_start, a.big_tiles,
                     a.status);
  if (a.n_tiles > 0) {            // 2 .. 512 keys: one wave per list; .. 2048: 2 or 4 waves; .. 4096 (= kSortCap)
    // the longer classes walk the longest-first order (bounded grids where few lists are that long)
    unsigned long long* k = a.keys[a.sorted];
    const int nt = a.n_tiles;
    hipLaunchKernelGGL(k_sort_lists_wave, dim3((nt + 3) / 4), dim3(256), 0, s, k, a.tile_start,
                       a.tile_order, nt, a.status);
    hipLaunchKernelGGL(k_sort_lists_wg<2>, dim3(nt), dim3(128), 0, s, k, a.tile_start, a.tile_order,
                       nt, kWaveSortMax, a.status);
    hipLaunchKernelGGL(k_sort_lists_wg<4>, dim3(std::min(nt, 2048)), dim3(256), 0, s, k, a.tile_start, a.tile_order,
                       nt, 2 * kWaveSortMax, a.status);
    hipLaunchKernelGGL((k_sort_blocks<512, 8>), dim3(std::min(nt, 256)), dim3(512), 0, s, k, a.tile_start,
                       a.tile_order, nt, kWgSortMax, a.status);
  }
}

hipError_t launch_bin_view(BinArgs& a, hipStream_t s) {
  const int nb = (int)((a.n + 255) / 256);
  if (a.n > 0) {
    StageTimer::begin(kStProject, s);
    hipLaunchKernelGGL(k_project, dim3(nb), dim3(256), 0, s, a.means, a.log_scales, a.quats, a.opacities,
                       a.n, a.cam, a.tile_shift, a.splats, a.offsets);
    StageTimer::end(kStProject, s);
  }
  StageTimer::begin(kStScan, s);
  const int sb = (int)scan_blocks(a.n);
  if (sb > 0)
    hipLaunchKernelGGL(k_scan_reduce, dim3(sb), dim3(256), 0, s, a.offsets, a.n, a.scan_part);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, a.scan_part, sb,
                     (unsigned long long)a.capacity, a.status);
  if (sb > 0)
    hipLaunchKernelGGL(k_scan_down, dim3(sb), dim3(256), 0, s, a.offsets, a.n, a.scan_part, a.offsets + a.n);
  StageTimer::end(kStScan, s);
  const bool counting = a.bin_hist && count_binning_ok(a.n, a.n_tiles);
  if (a.n > 0 && !counting) {
    StageTimer::begin(kStEmit, s);
    hipLaunchKernelGGL(k_emit, dim3(nb), dim3(256), 0, s, a.splats, a.n, a.tiles_x, a.n_tiles, a.tile_shift,
                       a.cam.width, a.cam.height, (const unsigned int*)a.offsets, a.tile_ids[0], a.keys[0],
                       (a.n_cull_records > 0 || a.pair_index) ? 1 : 0, a.status);
    StageTimer::end(kStEmit, s);
  }
  StageTimer::begin(kStSortBig, s);
  if (a.n_cull_records > 0 && a.n > 0)
    hipLaunchKernelGGL(k_clear_records, dim3(1024), dim3(256), 0, s, cull_of(a), (const Status*)a.status);
  if (counting) {
    const int nwg = count_groups(a.n);
    const long long per_wg = std::max<long long>(1, (a.n + nwg - 1) / nwg);
    const size_t lds = sizeof(unsigned int) * (size_t)((a.n_tiles + 1) / 2);
    hipLaunchKernelGGL(k_bin_count, dim3(nwg), dim3(kCountThreads), lds, s, a.splats, a.n, a.tiles_x, a.n_tiles,
                       a.tile_shift, a.cam.width, a.cam.height, per_wg, a.bin_hist, a.status);
    const int cst = colscan_tiles_per_wg(nwg);
    hipLaunchKernelGGL(k_bin_colscan, dim3((a.n_tiles + cst - 1) / cst), dim3(256), 0, s, a.bin_hist, nwg,
                       a.n_tiles, a.tile_start, a.status);
    launch_tile_scan_order(a, s);
    const size_t lds_place = lds + (a.n_tiles <= kCountPlaceLdsTiles ? sizeof(unsigned int) * (size_t)a.n_tiles : 0);
    hipLaunchKernelGGL(k_bin_place, dim3(nwg), dim3(kCountThreads), lds_place, s,
                       a.splats, a.n, a.tiles_x, a.n_tiles,
                       a.tile_shift, a.cam.width, a.cam.height, per_wg, (const unsigned int*)a.bin_hist,
                       (const unsigned int*)a.tile_start, a.keys[0],
                       (a.n_cull_records > 0 || a.pair_index) ? (const unsigned int*)a.offsets : nullptr, a.status);
    a.sorted = 0;
    sort_lists(a, s, true);
    StageTimer::end(kStSortBig, s);
    return hipGetLastError();
  }
  // radix sort by tile id: passes alternate between the two buffers
  const int passes = radix_passes(a.n_tiles + 1);   // tile ids 0..n_tiles (n_tiles: unreachable block)
  const int rb = (int)radix_blocks(a.capacity);
  const long long hlen = (long long)rb * kRadixBins;
  const int hsb = (int)scan_blocks(hlen);
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(rb), dim3(256), 0, s, a.tile_ids[cur], shift, rb, a.radix_hist,
                       a.status);
    hipLaunchKernelGGL(k_scan_reduce, dim3(hsb), dim3(256), 0, s, a.radix_hist, hlen, a.scan_part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, a.scan_part, hsb, 0ull, (Status*)nullptr);
    hipLaunchKernelGGL(k_scan_down, dim3(hsb), dim3(256), 0, s, a.radix_hist, hlen, a.scan_part,
                       (unsigned int*)nullptr);
    hipLaunchKernelGGL(k_radix_scatter, dim3(rb), dim3(256), 0, s, a.tile_ids[cur], a.keys[cur], shift, rb,
                       a.radix_hist, a.tile_ids[cur ^ 1], a.keys[cur ^ 1], a.status);
    cur ^= 1;
  }
  a.sorted = cur;
  hipLaunchKernelGGL(k_tile_ranges, dim3((a.n_tiles + 1 + 255) / 256), dim3(256), 0, s, a.tile_ids[cur],
                     a.n_tiles, a.tile_start, a.sort_cap, a.big_tiles, a.status);
  sort_lists(a, s, false);
  StageTimer::end(kStSortBig, s);
  return hipGetLastError();
}

}  // namespace scoup
