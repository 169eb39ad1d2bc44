// Uplift path of libscoup: projection, tile binning, per-tile depth sort,
// front-to-back compositing fused with the weighted sparse accumulation, and
// the per-row Top-K filter.  gfx950 (CDNA4), wave64.
//
// Paper mapping:
//   k_project        Sec. 3 (3DGS Gaussians, EWA splat of the tile rasterizer
//                    that produces alpha_i = o_i G_i^2D of Eq. 2)
//   k_tile_scan,
//   k_emit, sort     tile binning and front-to-back order of N_{v,p} (Eq. 1)
//   k_composite_acc  Eq. 2 weights e = alpha T, then Eq. 5 / Algorithm 1:
//                    w_i[j] += c_j e_i(v,p) for each code slot of the pixel's region
//   k_topk           Eq. 6 Top-K and L1 normalisation
#include <hip/hip_runtime.h>
#include <math.h>

#include "scoup_device.h"
#include "scoup_internal.h"

namespace scoup {

// ---------------------------------------------------------------------------
// projection (one thread per Gaussian), FP64 arithmetic, FP32 storage
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_project(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ opacities, long long n,
    CamDev cam, int tiles_x, int tile_shift, GSplat* __restrict__ out,
    unsigned int* __restrict__ tile_count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  GSplat s;
  s.ix = 0; s.iy = 0; s.fx = 0.f; s.fy = 0.f;
  s.l00 = 0.f; s.l10 = 0.f; s.l11 = 0.f; s.opacity = 0.f;
  s.bx0 = 1; s.bx1 = 0; s.by0 = 1; s.by1 = 0;   // empty box = invisible
  s.depth_bits = 0u; s.pad = 0u;

  const double mx = means[3 * i + 0], my = means[3 * i + 1], mz = means[3 * i + 2];
  double x, y, z;
  {
    // Camera point p = R mu + t summed left to right without fused multiply-adds,
    // so the view depth (and its float32 sort key) is reproducible exactly.
#pragma clang fp contract(off)
    x = (double)cam.R[0] * mx + (double)cam.R[1] * my + (double)cam.R[2] * mz + (double)cam.t[0];
    y = (double)cam.R[3] * mx + (double)cam.R[4] * my + (double)cam.R[5] * mz + (double)cam.t[1];
    z = (double)cam.R[6] * mx + (double)cam.R[7] * my + (double)cam.R[8] * mz + (double)cam.t[2];
  }
  const double o = opacities[i];
  const double lo = log(255.0 * o);
  if (!(z > (double)cam.near_z) || !(lo >= 0.0)) { out[i] = s; return; }

  // 3D covariance Sigma = R diag(exp(2 s)) R^T from the normalised quaternion
  double qw = quats[4 * i + 0], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
  const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const double Rq[3][3] = {
      {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
      {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
      {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
  const double s2[3] = {exp(2.0 * (double)log_scales[3 * i + 0]),
                        exp(2.0 * (double)log_scales[3 * i + 1]),
                        exp(2.0 * (double)log_scales[3 * i + 2])};
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
  if (!(det > 0.0) || !(fabs(mux) < 1073741824.0) || !(fabs(muy) < 1073741824.0)) {
    out[i] = s; return;
  }
  // conservative pixel box of {alpha >= 1/255}: |dx| <= sqrt(2 ln(255 o) Sxx)
  const double r2 = 2.0 * lo;
  const double hx = sqrt(r2 * sxx), hy = sqrt(r2 * syy);
  double x0 = ceil(mux - hx - 0.5) - 1.0, x1 = floor(mux + hx - 0.5) + 1.0;
  double y0 = ceil(muy - hy - 0.5) - 1.0, y1 = floor(muy + hy - 0.5) + 1.0;
  x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
  x1 = fmin(x1, (double)(cam.width - 1)); y1 = fmin(y1, (double)(cam.height - 1));
  if (!(x0 <= x1) || !(y0 <= y1)) { out[i] = s; return; }

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
  out[i] = s;
  const int tx0 = s.bx0 >> tile_shift, tx1 = s.bx1 >> tile_shift;
  const int ty0 = s.by0 >> tile_shift, ty1 = s.by1 >> tile_shift;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&tile_count[ty * tiles_x + tx], 1u);
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-tile counts (one workgroup), capacity check
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_tile_scan(unsigned int* __restrict__ tile_count,
                                                    unsigned int* __restrict__ tile_cursor,
                                                    unsigned int* __restrict__ tile_start, int nt,
                                                    unsigned long long capacity, Status* st) {
  __shared__ unsigned long long part[1024];
  const int tid = threadIdx.x;
  const int per = (nt + 1023) / 1024;
  const int b = tid * per, e = min(nt, b + per);
  unsigned long long sum = 0;
  for (int t = b; t < e; ++t) sum += tile_count[t];
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // Hillis-Steele inclusive scan
    unsigned long long v = tid >= o ? part[tid - o] : 0ull;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  unsigned long long run = part[tid] - sum;
  const unsigned long long total = part[1023];
  const bool over = total > capacity;
  for (int t = b; t < e; ++t) {
    const unsigned int c = tile_count[t];
    tile_start[t] = over ? 0u : (unsigned int)run;
    run += c;
    tile_count[t] = 0u;       // ready for the next view
    tile_cursor[t] = 0u;
  }
  if (tid == 0) {
    tile_start[nt] = over ? 0u : (unsigned int)total;
    st->total_pairs = over ? 0u : (unsigned int)total;
    st->view_overflow = over ? 1u : 0u;
    const unsigned int tot32 = total > 0xffffffffull ? 0xffffffffu : (unsigned int)total;
    if (over) st->any_overflow = 1u;
    if (tot32 > st->max_pairs) st->max_pairs = tot32;
  }
}

// ---------------------------------------------------------------------------
// emit one (depth, id) key per (Gaussian, tile) into the tile's bucket
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_emit(const GSplat* __restrict__ splats, long long n,
                                              int tiles_x, int tile_shift,
                                              const unsigned int* __restrict__ tile_start,
                                              unsigned int* __restrict__ tile_cursor,
                                              unsigned long long* __restrict__ keys, const Status* st) {
  if (st->view_overflow) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GSplat s = splats[i];
  if (s.bx0 > s.bx1) return;
  const unsigned long long key = ((unsigned long long)s.depth_bits << 32) | (unsigned long long)i;
  const int tx0 = s.bx0 >> tile_shift, tx1 = s.bx1 >> tile_shift;
  const int ty0 = s.by0 >> tile_shift, ty1 = s.by1 >> tile_shift;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      const int t = ty * tiles_x + tx;
      const unsigned int pos = atomicAdd(&tile_cursor[t], 1u);
      keys[tile_start[t] + pos] = key;
    }
}

// Tiles whose list exceeds the LDS capacity are sorted in place in global
// memory by one workgroup (rare; correctness path for dense tiles).
__global__ __launch_bounds__(1024) void k_sort_big(unsigned long long* __restrict__ keys,
                                                   const unsigned int* __restrict__ tile_start,
                                                   int sort_cap, const Status* st) {
  if (st->view_overflow) return;
  const int tile = blockIdx.x;
  const unsigned int start = tile_start[tile];
  const long long L = (long long)tile_start[tile + 1] - start;
  if (L <= sort_cap) return;
  unsigned long long* s = keys + start;
  long long n2 = 1;
  while (n2 < L) n2 <<= 1;
  const int tid = threadIdx.x;
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
}

// ---------------------------------------------------------------------------
// composite + weighted sparse accumulate, one 16x16 tile per workgroup;
// wave w owns the 8x8 quadrant (w&1, w>>1), lane l pixel (l&7, l>>3) of it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_composite_acc(
    const GSplat* __restrict__ splats, const unsigned int* __restrict__ tile_start,
    const unsigned long long* __restrict__ keys, int tiles_x, int W, int H,
    const int* __restrict__ rmap, int n_regions, long long region_base,
    const int* __restrict__ code_idx, const float* __restrict__ code_val, int k_code,
    int m_atoms, float* __restrict__ acc, Status* st) {
  __shared__ unsigned long long s_keys[kSortCap];
  __shared__ GSplat s_g[kTileThreads];
  __shared__ unsigned int s_id[kTileThreads];
  if (st->view_overflow) return;
  const int tile = blockIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const unsigned int start = tile_start[tile];
  const int L = (int)(tile_start[tile + 1] - start);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int qx = (wave & 1) * 8, qy = (wave >> 1) * 8;
  const int lx = qx + (lane & 7), ly = qy + (lane >> 3);
  const int tile_x0 = tx * kTile, tile_y0 = ty * kTile;
  const int px = tile_x0 + lx, py = tile_y0 + ly;
  const bool inside = px < W && py < H;
  int reg = -1;
  if (inside) {
    reg = rmap[(long long)py * W + px];
    if (reg < -1 || reg >= n_regions) { atomicOr(&st->data_error, 1u); reg = -1; }
  }
  if (L == 0) return;   // region ids are validated on every pixel, empty tiles included
  const int qx0 = tile_x0 + qx, qx1 = qx0 + 7, qy0 = tile_y0 + qy, qy1 = qy0 + 7;
  const float pcx = (float)lx + 0.5f, pcy = (float)ly + 0.5f;

  const bool in_lds = L <= kSortCap;
  if (in_lds) {
    int n2 = 1;
    while (n2 < L) n2 <<= 1;
    for (int j = tid; j < n2; j += kTileThreads) s_keys[j] = j < L ? keys[start + j] : ~0ull;
    __syncthreads();
    bitonic_lds(s_keys, n2, tid, kTileThreads);
  }

  float T = 1.0f;
  bool done = !inside;
  unsigned long long count = 0;
  for (int b0 = 0; b0 < L; b0 += kTileThreads) {
    if (__syncthreads_count(!done) == 0) break;
    const int j = b0 + tid;
    if (j < L) {
      const unsigned long long k = in_lds ? s_keys[j] : keys[start + j];
      const unsigned int id = (unsigned int)k;
      s_id[tid] = id;
      s_g[tid] = splats[id];
    }
    __syncthreads();
    const int nb = min(kTileThreads, L - b0);
    if (__ballot(!done) != 0ull) {
      for (int k = 0; k < nb; ++k) {
        const GSplat g = s_g[k];
        if (g.bx1 < qx0 || g.bx0 > qx1 || g.by1 < qy0 || g.by0 > qy1) continue;
        const float hx = (float)(g.ix - tile_x0), hy = (float)(g.iy - tile_y0);
        const float dx = (pcx - hx) - g.fx, dy = (pcy - hy) - g.fy;
        const float u = fmaf(g.l00, dx, g.l10 * dy), v = g.l11 * dy;
        const float q = fmaf(u, u, v * v);
        const float alpha = fminf(kAlphaMax, g.opacity * __builtin_amdgcn_exp2f(-q));
        const bool take = !done && alpha >= kAlphaMin;
        if (__ballot(take) == 0ull) continue;
        float e = 0.0f;
        if (take) {
          const float testT = T * (1.0f - alpha);
          if (testT < kTMin) {
            done = true;
          } else {
            e = alpha * T;
            T = testT;
          }
        }
        const unsigned long long cm = __ballot(e > 0.0f);
        if (cm) {
          count += (unsigned long long)__popcll(cm);
          unsigned long long rm = __ballot(e > 0.0f && reg >= 0);
          const unsigned long long row = (unsigned long long)s_id[k] * (unsigned long long)m_atoms;
          while (rm) {
            const int l0 = __ffsll((long long)rm) - 1;
            const int r0 = __shfl(reg, l0, 64);
            const unsigned long long same = __ballot(reg == r0) & rm;
            const float sum = wave_sum(((same >> lane) & 1ull) ? e : 0.0f);
            const long long gr = (region_base + r0) * (long long)k_code;
            for (int c = lane; c < k_code; c += 64) {
              const int jj = code_idx[gr + c];
              if (jj >= m_atoms) atomicOr(&st->data_error, 2u);
              else if (jj >= 0) atomic_add_f32(&acc[row + (unsigned long long)jj], sum * code_val[gr + c]);
            }
            rm &= ~same;
          }
        }
        if (__ballot(!done) == 0ull) break;
      }
    }
    __syncthreads();
  }
  if (lane == 0 && count) atomicAdd(&st->contrib, count);
}

// ---------------------------------------------------------------------------
// Top-K per row (one wave per row), Eq. 6
// ---------------------------------------------------------------------------
template <int NS>
__global__ __launch_bounds__(256) void k_topk(const float* __restrict__ acc, long long n, int m, int k,
                                              int* __restrict__ out_idx, float* __restrict__ out_val) {
  const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const float* a = acc + row * (long long)m;
  unsigned long long key[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int j = s * 64 + lane;
    const float v = j < m ? a[j] : 0.0f;
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
    out_idx[row * k + lane] = sel_i;
    out_val[row * k + lane] = sel_i >= 0 ? sel_v / sum : 0.0f;
  }
}

__global__ void k_add_u64(unsigned long long* dst, const Status* st) { *dst += st->contrib; }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_bin_view(const BinArgs& a, hipStream_t s) {
  const int nb = (int)((a.n + 255) / 256);
  if (a.n > 0) {
    StageTimer::begin(kStProject, s);
    hipLaunchKernelGGL(k_project, dim3(nb), dim3(256), 0, s, a.means, a.log_scales, a.quats,
                       a.opacities, a.n, a.cam, a.tiles_x, a.tile_shift, a.splats, a.tile_count);
    StageTimer::end(kStProject, s);
  }
  StageTimer::begin(kStScan, s);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, a.tile_count, a.tile_cursor,
                     a.tile_start, a.n_tiles, (unsigned long long)a.capacity, a.status);
  StageTimer::end(kStScan, s);
  if (a.n > 0) {
    StageTimer::begin(kStEmit, s);
    hipLaunchKernelGGL(k_emit, dim3(nb), dim3(256), 0, s, a.splats, a.n, a.tiles_x, a.tile_shift,
                       a.tile_start, a.tile_cursor, a.keys, a.status);
    StageTimer::end(kStEmit, s);
  }
  StageTimer::begin(kStSortBig, s);
  hipLaunchKernelGGL(k_sort_big, dim3(a.n_tiles), dim3(1024), 0, s, a.keys, a.tile_start, a.sort_cap,
                     a.status);
  StageTimer::end(kStSortBig, s);
  return hipGetLastError();
}

hipError_t launch_uplift_view(const UpliftViewArgs& a, hipStream_t s) {
  hipError_t e = launch_bin_view(a.bin, s);
  if (e != hipSuccess) return e;
  const BinArgs& b = a.bin;
  StageTimer::begin(kStComposite, s);
  hipLaunchKernelGGL(k_composite_acc, dim3(b.n_tiles), dim3(kTileThreads), 0, s, b.splats,
                     b.tile_start, b.keys, b.tiles_x, b.cam.width, b.cam.height, a.rmap, a.n_regions,
                     a.region_base, a.code_idx, a.code_val, a.k_code, a.m_atoms, a.acc, b.status);
  StageTimer::end(kStComposite, s);
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
