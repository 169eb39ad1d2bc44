/*
 * scoup.h -- C ABI of libscoup, the MI355X (gfx950) implementation of the
 * sparse-code uplift, sparse coefficient render and codebook decode of
 * "Sparse Code Uplifting for Efficient 3D Language Gaussian Splatting" (SCOUP).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments marked "device" are device pointers owned by the
 *   caller (HIP allocations on the current device).  Arrays marked "host"
 *   live in host memory and are only read during the call.
 * - The library never allocates device memory.  Scratch space comes from the
 *   caller's workspace `ws` of `ws_bytes` bytes (device, 256-byte aligned),
 *   sized with the matching *_workspace_bytes query.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *   enqueued on it; every call returns after a single device->host read of a
 *   small status block on that stream (so results are complete on return).
 * - Arguments are validated on the host before any launch; a non-OK status
 *   leaves outputs unspecified and sets a thread-local message that
 *   scoup_last_error() returns.
 * - Floating-point results are float32; weight and coefficient accumulation
 *   is float32 everywhere.  Atomic float additions make bit-level results
 *   depend on scheduling (sums are order-dependent at the 1e-7 level).
 */
#ifndef SCOUP_H_
#define SCOUP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCOUP_OK = 0,
  SCOUP_E_ARG = -1,          /* invalid argument (null pointer, bad size, K > M ...) */
  SCOUP_E_WORKSPACE = -2,    /* workspace too small; see scoup_required_pair_capacity() */
  SCOUP_E_HIP = -3,          /* a HIP runtime call failed */
  SCOUP_E_UNSUPPORTED = -4,  /* valid but unsupported configuration */
  SCOUP_E_DATA = -5          /* bad data found on the device (region id out of range) */
} scoup_status;

typedef enum { SCOUP_F32 = 0, SCOUP_BF16 = 1, SCOUP_FP8_E4M3 = 2 } scoup_dtype;

/* 3D Gaussians (Sec. 3 "Preliminaries": centre mu, scale s, rotation q,
 * opacity o; the view-dependent colour is not used).  Structure of arrays,
 * device, float32:
 *   means      [n*3]  world-space centres
 *   log_scales [n*3]  per-axis log standard deviations (activation exp)
 *   quats      [n*4]  rotation quaternions (w,x,y,z), normalised by the library
 *   opacities  [n]    activated opacities in (0,1)                          */
typedef struct {
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacities;
} scoup_gaussians;

/* Pinhole camera (host).  World point X maps to camera point R X + t
 * (R row-major, world->camera); camera axes +x right, +y down, +z forward;
 * pixel coordinates (fx x/z + cx, fy y/z + cy); pixel (px,py) is sampled at
 * its centre (px+0.5, py+0.5).  Points with z <= near_z are culled.         */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float near_z;
} scoup_camera;

/* The per-view inputs of the uplift (Sec. 4.1-4.2, Algorithm 1).
 *   cams         host [n_views]
 *   region_maps  device int32, the H_v*W_v maps of all views concatenated
 *                row-major; value r >= 0 is a view-local region id, -1 = no
 *                region (the pixel composites but carries no code)
 *   map_offsets  host [n_views+1], element offset of each view's map
 *   region_base  host [n_views+1]; view v has region_base[v+1]-region_base[v]
 *                regions and region r of view v has global id region_base[v]+r
 *   code_idx     device int32 [R_total*k_code] atom index of each code slot,
 *                -1 = empty slot
 *   code_val     device float32 [R_total*k_code] coefficient of each slot
 *                (Eq. 4: non-negative, summing to one; not checked)
 *   k_code       slots per region code (K of Eq. 4)
 *   m_atoms      codebook size (L of Eq. 4, "M" in this library)          */
typedef struct {
  int32_t n_views;
  const scoup_camera* cams;
  const int32_t* region_maps;
  const int64_t* map_offsets;
  const int64_t* region_base;
  const int32_t* code_idx;
  const float* code_val;
  int32_t k_code;
  int32_t m_atoms;
} scoup_views;

/* Workspace bytes for scoup_uplift / scoup_uplift_accumulate.
 *   pair_capacity  capacity for (Gaussian, 8x8-block) pairs of one view
 *                  (0 picks 6 pairs per Gaussian)
 *   view_batch     views whose per-pair records are kept before they are summed
 *                  into the accumulator (0 = all views: one pass over acc)
 * The workspace holds, per view of a batch, (n+1) pair offsets and two 8-byte
 * region records per pair, plus one view's projected splats and sort buffers
 * (about n*52 + pair_capacity*(24.25 + 16*view_batch) + 4*(n+1)*view_batch bytes). */
size_t scoup_uplift_workspace_bytes(int64_t n_gaussians, const scoup_views* views,
                                    int64_t pair_capacity, int32_t view_batch);

/* After SCOUP_E_WORKSPACE: the pair capacity the failed call needed (the
 * largest per-view pair count it saw).  Thread-local.                       */
int64_t scoup_required_pair_capacity(void);

/* Weighted sparse accumulation, Eq. 5 without the normaliser Z_i (Eq. 6
 * subsumes it) and the loops of Algorithm 1:
 *   acc[i*m + j] += sum over views v, pixels p with region r >= 0,
 *                   Gaussians i in N_{v,p}, code slots (j, c) of region r:
 *                   c * e_i(v,p)
 * with e_i(v,p) = alpha_i T_i the front-to-back blending weight of Eq. 2 under
 * the 3DGS numerics (alpha = min(0.99, o G2D); alpha < 1/255 skipped; the
 * Gaussian that would take T below 1e-4 is excluded and ends the pixel),
 * G2D the EWA splat with +0.3 px^2 dilation and the 1.3 tan(fov/2) Jacobian
 * clamp, depth order by float32(view depth) with ties to the lower index.
 *   acc           device float32 [n*m], row-major (Gaussian-major)
 *   accumulate    0: acc is overwritten (zeroed first); 1: results are added to
 *                 the values already in acc (resume over a further view set)
 *   pair_capacity, view_batch  as given to scoup_uplift_workspace_bytes
 *   ws, ws_bytes  at least scoup_uplift_workspace_bytes(n, views, pair_capacity, view_batch)
 *   n_contrib     device uint64 [1] or NULL; receives (+=) the number of
 *                 Gaussian-pixel contributions (terms e > 0) composited
 * Returns SCOUP_E_WORKSPACE if the workspace is too small or a view's pair
 * count exceeds pair_capacity (call again with scoup_required_pair_capacity()),
 * SCOUP_E_DATA if a region id is >= the view's region count or a code atom
 * index is >= m.  After SCOUP_E_WORKSPACE with accumulate = 0, acc holds
 * unspecified values (a successful call overwrites it); with accumulate = 1
 * every view's pair count is checked before anything is written (one more
 * pass over the Gaussians per 32 views), so acc is left unchanged and the
 * same call can simply be repeated with a larger capacity.  After
 * SCOUP_E_DATA acc is unspecified in both modes.                            */
scoup_status scoup_uplift_accumulate(const scoup_gaussians* g, const scoup_views* views,
                                     float* acc, int32_t accumulate, int64_t pair_capacity,
                                     int32_t view_batch, void* ws, size_t ws_bytes,
                                     unsigned long long* n_contrib, void* stream);

/* Top-K filter and L1 normalisation of Eq. 6, per row of acc (n rows of m):
 * entries ranked by (value descending, index ascending); the first k strictly
 * positive ones are kept and divided by their sum; missing entries are padded
 * with (idx -1, val 0); an all-zero row is all padding (Algorithm 1 skips it).
 *   acc      device float32 [n*m]   (read only)
 *   idx      device int32   [n*k]   atom indices in rank order
 *   val      device float32 [n*k]   normalised coefficients
 * Requires 1 <= k <= m <= 4096.                                             */
scoup_status scoup_topk(const float* acc, int64_t n, int32_t m, int32_t k,
                        int32_t* idx, float* val, void* stream);

/* Dense feature uplift, Eq. 3 (the baseline the sparse uplift replaces):
 *   features[i*dim + d] = (1/Z_i) sum over (v,p) with region r >= 0 of
 *                         e_i(v,p) F_r[d],  F_r = sum over code slots c C[j]   (Eq. 4)
 *   z[i] = Z_i = sum of those e_i(v,p)    (rows with Z_i = 0 are zero)
 * Same compositing as scoup_uplift; each (Gaussian, region) weight adds a
 * dim-wide feature instead of k_code coefficients.
 *   codebook  device float32 [m_atoms*dim];  features device float32 [n*dim];
 *   z device float32 [n]; 1 <= dim <= 1024.  Workspace from
 *   scoup_uplift_dense_workspace_bytes (adds R_total*dim floats).          */
size_t scoup_uplift_dense_workspace_bytes(int64_t n_gaussians, const scoup_views* views, int32_t dim,
                                          int64_t pair_capacity, int32_t view_batch);
scoup_status scoup_uplift_dense(const scoup_gaussians* g, const scoup_views* views, const float* codebook,
                                int32_t dim, float* features, float* z, int64_t pair_capacity,
                                int32_t view_batch, void* ws, size_t ws_bytes,
                                unsigned long long* n_contrib, void* stream);

/* Entropy of each Gaussian's coefficient distribution (App. C.2):
 * out[i] = -sum_j p_j log p_j with p = acc row i / its sum over positive
 * entries (natural log, 0 log 0 = 0), 0 for an all-zero row.
 *   acc  device float32 [n*m] (read only);  out  device float32 [n]        */
scoup_status scoup_entropy(const float* acc, int64_t n, int32_t m, float* out, void* stream);

/* The full uplift of Algorithm 1: acc is zeroed, accumulated over every view
 * and reduced to k coefficients per Gaussian (Eq. 6, as scoup_topk; fused
 * into the last accumulation pass).  Requires 1 <= k <= min(64, m) and
 * m <= 4096.  Other arguments as scoup_uplift_accumulate.                   */
scoup_status scoup_uplift(const scoup_gaussians* g, const scoup_views* views, int32_t k,
                          float* acc, int32_t* topk_idx, float* topk_val, int64_t pair_capacity,
                          int32_t view_batch, void* ws, size_t ws_bytes,
                          unsigned long long* n_contrib, void* stream);

/* ---------------------------------------------------------------------------
 * Sparse coefficient render (Eq. 7), decode (Eq. 8) and their backward
 * ------------------------------------------------------------------------- */

/* Workspace bytes for scoup_render_coeff on `cam` given a capacity for
 * (Gaussian, 8x8-block) pairs; 0 picks 16 pairs per Gaussian.               */
size_t scoup_render_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam,
                                    int64_t pair_capacity);

/* Eq. 7 for one camera: coeff_map[p*m + j] = coeff_scale * sum over Gaussians i
 * in N_{v,p} (same compositing as the uplift) of e_i(v,p) * topk_val[i*k + s]
 * for every slot s with topk_idx[i*k + s] == j (slots with index -1 are
 * skipped).  The products e * topk_val are float32 and are summed in float32
 * on the matrix cores, two Gaussians at a time in the block's front-to-back
 * list order (a fixed order: bit-reproducible); the map is written once per pixel in
 * coeff_dtype (F32, BF16 round-to-nearest-even, or FP8 E4M3 saturating; use
 * coeff_scale to place FP8 values in range, e.g. 256 since coefficients are
 * at most 1).
 *   topk_idx   device int32   [n*k], 1 <= k <= 16, n*k < 2^30, indices < m_atoms (else SCOUP_E_DATA)
 *   topk_val   device float32 [n*k]
 *   coeff_map  device [H*W*m_atoms] of coeff_dtype, pixel-major (y*W + x)
 *   t_final    device float32 [H*W] transmittance left at each pixel, or NULL
 *   n_contrib  device uint64 [1] (+=) contributions composited, or NULL
 * Requires 1 <= m_atoms <= 512 (64 pixel rows of m_atoms floats in LDS).    */
scoup_status scoup_render_coeff(const scoup_gaussians* g, const int32_t* topk_idx,
                                const float* topk_val, int32_t k, int32_t m_atoms,
                                const scoup_camera* cam, void* coeff_map, scoup_dtype coeff_dtype,
                                float coeff_scale, float* t_final, void* ws, size_t ws_bytes,
                                unsigned long long* n_contrib, void* stream);

/* Workspace bytes for scoup_render: the codebook converted to in_dtype in
 * MFMA operand order, then scoup_render_workspace_bytes(n, cam, pair_capacity)
 * (0 picks 8 pairs per Gaussian).                                           */
size_t scoup_render_decode_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam, int32_t m_atoms,
                                           int32_t dim, scoup_dtype in_dtype, int64_t pair_capacity);

/* The render of Sec. 4.3 in one pass: Eq. 7 and then Eq. 8 for one camera,
 *   features[p*dim + d] = sum_j W_hat(p)[j] codebook[j*dim + d]
 * with W_hat(p) the float32 coefficient row of scoup_render_coeff, kept on
 * chip per 8x8 pixel block and multiplied by the codebook on MFMA (float32
 * accumulation) before the next block: the P x m map never reaches memory
 * unless coeff_map asks for it.  in_dtype is the precision of that product:
 * F32; BF16 (rows and codebook rounded to nearest even); FP8 E4M3 (rows times
 * 256, codebook times a power-of-two scale, both divided out in float32).
 * With in_dtype F32, or whenever coeff_map is given, the rows are those of
 * scoup_render_coeff and the features equal scoup_decode applied to the
 * scoup_render_coeff map of the same precision (F32 map, BF16 map, FP8 map
 * with coeff_scale 256), bit for bit.  BF16 / FP8 without coeff_map sum the
 * rows from bfloat16-rounded products e * topk_val instead (one bfloat16
 * rounding per term; the result is still bit-reproducible).  Pixels without a
 * contribution get zero features.
 *   topk_idx/val   device [n*k], 1 <= k <= 16, n*k < 2^30, indices < m_atoms (else SCOUP_E_DATA)
 *   codebook       device float32 [m_atoms*dim], 1 <= m_atoms <= 512, 1 <= dim <= 1024
 *   coeff_map      device float32 [H*W*m_atoms] (the float32 W_hat, as for the
 *                  backward), or NULL
 *   t_final        device float32 [H*W] transmittance left at each pixel, or NULL
 *   features       device [H*W*dim] of out_dtype (F32 or BF16, round to nearest even)
 *   ws, ws_bytes   at least scoup_render_decode_workspace_bytes(...); the pair
 *                  capacity is what remains after the converted codebook
 *   n_contrib      device uint64 [1] (+=) contributions composited, or NULL
 * Returns SCOUP_E_WORKSPACE when the view has more (Gaussian, block) pairs
 * than the workspace holds (scoup_required_pair_capacity() gives the count). */
scoup_status scoup_render(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val, int32_t k,
                          const scoup_camera* cam, const float* codebook, int32_t m_atoms, int32_t dim,
                          scoup_dtype in_dtype, float* coeff_map, float* t_final, void* features,
                          scoup_dtype out_dtype, void* ws, size_t ws_bytes, unsigned long long* n_contrib,
                          void* stream);

/* Workspace bytes for scoup_render_views over n_views cameras of cam's image
 * size: the converted codebook once, then one scoup_render_workspace_bytes
 * set of binning buffers per view in flight (min(4, n_views) sets).        */
size_t scoup_render_views_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam, int32_t n_views,
                                          int32_t m_atoms, int32_t dim, scoup_dtype in_dtype,
                                          int64_t pair_capacity);

/* scoup_render (Sec. 4.3, Eq. 7 then Eq. 8) for n_views cameras of one image
 * size, without a coefficient map or t_final: view v's features are exactly
 * those scoup_render gives for cams[v] with coeff_map NULL, bit for bit.  Up
 * to scoup_views_in_flight() views run at once (view v on the caller's stream
 * or one of the library's streams, each with its own binning buffers), so
 * the projection and binning of one view overlap the render kernel of
 * another; the call returns after every view is done.
 *   cams           host [n_views], every camera of cams[0]'s width and height
 *                  (else SCOUP_E_ARG)
 *   features       device [n_views*H*W*dim] of out_dtype, view-major
 *   ws, ws_bytes   at least scoup_render_views_workspace_bytes(...); each set
 *                  gets an equal share of what remains after the codebook
 *   n_contrib      device uint64 [1] (+=) contributions of all views, or NULL
 * Other arguments and limits as scoup_render.  Returns SCOUP_E_WORKSPACE when
 * a view has more pairs than a set holds (scoup_required_pair_capacity()
 * gives the largest count); the features are then incomplete.             */
scoup_status scoup_render_views(const scoup_gaussians* g, const int32_t* topk_idx, const float* topk_val, int32_t k,
                                const scoup_camera* cams, int32_t n_views, const float* codebook, int32_t m_atoms,
                                int32_t dim, scoup_dtype in_dtype, void* features, scoup_dtype out_dtype, void* ws,
                                size_t ws_bytes, unsigned long long* n_contrib, void* stream);

/* Workspace bytes for scoup_decode (the codebook converted to in_dtype and
 * arranged in MFMA operand order).                                          */
size_t scoup_decode_workspace_bytes(int32_t m_atoms, int32_t dim, scoup_dtype in_dtype);

/* Eq. 8: features[p*dim + d] = (1/coeff_scale) sum_j coeff[p*m + j] * codebook[j*dim + d]
 * on MFMA with float32 accumulation.  The float32 codebook is converted to
 * in_dtype inside the call (FP8 with a power-of-two per-tensor scale that is
 * divided out again).  out_dtype is F32 or BF16 (round to nearest even).
 *   coeff     device [n_pixels*m_atoms] of in_dtype
 *   codebook  device float32 [m_atoms*dim]
 *   features  device [n_pixels*dim] of out_dtype
 * Requires 1 <= m_atoms <= 4096 and 1 <= dim <= 1024.                       */
scoup_status scoup_decode(const void* coeff, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                          int32_t m_atoms, const float* codebook, int32_t dim, void* features,
                          scoup_dtype out_dtype, void* ws, size_t ws_bytes, void* stream);

/* scoup_decode for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation, arguments, kernels and results as scoup_decode, without
 * a workspace.  The converted codebook and its scale live in a fixed scratch
 * array of scoup_decode_noalloc_max_bytes() bytes (8 MiB) that the library
 * holds on each GPU it runs on until the process ends; codebooks whose
 * scoup_decode_workspace_bytes exceed it are rejected with SCOUP_E_ARG
 * (e.g. F32 up to m_atoms * dim of about 2M).  The call allocates nothing and
 * records no stage timing.  Every call on a GPU shares that GPU's scratch:
 * calls that overlap on one GPU (other threads, other streams) race and must
 * be serialised by the caller.  Returns after the work is complete, like
 * scoup_decode.                                                             */
size_t scoup_decode_noalloc_max_bytes(void);
scoup_status scoup_decode_noalloc(const void* coeff, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                                  int32_t m_atoms, const float* codebook, int32_t dim, void* features,
                                  scoup_dtype out_dtype, void* stream);

/* Workspace bytes for scoup_relevancy (the codebook folded into the query
 * and canonical vectors, in MFMA operand order).                            */
size_t scoup_relevancy_workspace_bytes(int32_t m_atoms, int32_t n_queries, scoup_dtype in_dtype);

/* Relevancy of App. B on the decoded features of Eq. 8, without writing them:
 *   scores[p*n_queries + q] = min over c < n_canon of
 *       1 / (1 + exp(temperature * (F(p).canon_c - F(p).query_q)))
 * with F(p) = (1/coeff_scale) coeff[p, :] codebook, i.e. the exponential
 * ratio of the appendix (temperature 10 there, 4 canonical phrases).  The
 * dot products are formed as coeff[p, :] (codebook query) with the folded
 * vectors computed in FP64; the per-pixel contraction runs on MFMA (float32
 * for F32 maps; bfloat16 with a two-term bfloat16 split of the folded vectors
 * for BF16 and FP8 maps), float32 accumulation and epilogue.
 *   coeff     device [n_pixels*m_atoms] of in_dtype (the map of scoup_render_coeff)
 *   codebook  device float32 [m_atoms*dim]
 *   queries   device float32 [n_queries*dim]
 *   canon     device float32 [n_canon*dim]
 *   scores    device float32 [n_pixels*n_queries] (coeff and scores may be NULL
 *             when n_pixels == 0)
 * Requires 1 <= m_atoms <= 4096, 1 <= dim <= 4096, 1 <= n_queries <= 1024,
 * 1 <= n_canon <= 4 and a finite temperature > 0 (else SCOUP_E_ARG).        */
scoup_status scoup_relevancy(const void* coeff, scoup_dtype in_dtype, float coeff_scale, int64_t n_pixels,
                             int32_t m_atoms, const float* codebook, int32_t dim, const float* queries,
                             int32_t n_queries, const float* canon, int32_t n_canon, float temperature,
                             float* scores, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for scoup_render_backward. */
size_t scoup_render_backward_workspace_bytes(int64_t n_gaussians, const scoup_camera* cam,
                                             int32_t m_atoms, int32_t dim, int64_t pair_capacity);

/* Backward of render + decode (float32) for a loss with gradient
 * G = dL/dfeatures on one camera (Eq. 7 and Eq. 8 differentiated):
 *   grad_codebook[j*dim + d] += sum_p coeff_map[p*m + j] G[p*dim + d]
 *   grad_topk_val[i*k + s]   += sum_p e_i(v,p) (G(p) C^T)[topk_idx[i*k + s]]
 * Indices and geometry receive no gradient.  coeff_map is the float32 map of
 * scoup_render_coeff (coeff_scale 1) for the same inputs.  Every sum is taken
 * in a fixed order (partial sums per pixel chunk and per (Gaussian, 8x8
 * block) pair, then added in order), so results are bit-reproducible.
 *   topk_idx/val   device [n*k], 1 <= k <= 16;  1 <= m_atoms <= 512;  1 <= dim <= 4096
 *   grad_features  device float32 [H*W*dim]
 *   grad_topk_val  device float32 [n*k]       (accumulated)
 *   grad_codebook  device float32 [m_atoms*dim] (accumulated)
 *   ws, ws_bytes   at least scoup_render_backward_workspace_bytes(n, cam, m_atoms,
 *                  dim, pair_capacity) (0 = 16 pairs per Gaussian); the pair
 *                  capacity is derived from ws_bytes
 * Returns SCOUP_E_WORKSPACE when the view has more (Gaussian, block) pairs
 * than the workspace holds (scoup_required_pair_capacity() gives the count);
 * the gradient buffers are then left unchanged.                             */
scoup_status scoup_render_backward(const scoup_gaussians* g, const int32_t* topk_idx,
                                   const float* topk_val, int32_t k, int32_t m_atoms,
                                   const scoup_camera* cam, const float* coeff_map,
                                   const float* codebook, int32_t dim, const float* grad_features,
                                   float* grad_topk_val, float* grad_codebook, void* ws,
                                   size_t ws_bytes, void* stream);

/* Optional per-stage kernel timing with HIP events recorded on the call's
 * stream around every launch (off by default; costs one event pair per
 * launch).  scoup_stage_timing(1) enables and resets the counters,
 * scoup_stage_timing(0) disables them.  scoup_stage_stats returns, for stage
 * id `stage`, the summed kernel time in milliseconds and the launch count
 * accumulated by completed calls since the last reset; it returns 0 on
 * success and -1 for an unknown stage.  Stage ids:
 *   0 project  1 pair scan  2 emit  3 tile sort  4 composite
 *   5 top-k    6 render     7 decode  8 render backward  9 backward GEMMs
 *   10 accumulator row build  11 relevancy  12 relevancy vector folding
 *   13 deferred further-region entries added to the accumulator
 * Process-wide state; not meant for concurrent calls from several threads. */
void scoup_stage_timing(int32_t enable);
int32_t scoup_stage_stats(int32_t stage, double* total_ms, int64_t* launches);

/* Statistics of the uplift calls completed while stage timing was enabled
 * (reset by scoup_stage_timing): the distinct (Gaussian, region) pairs of
 * level 0 that received a nonzero weight, summed over views -- U_v of the
 * byte model of Eq. 5's O(|S_i| K) cost, one code read per such pair.  Each
 * view's per-(Gaussian, block, region) records and deferred entries are
 * inserted into a hash set held in the view's sort buffer after the view is
 * composited (one more pass per view, statistics only).
 *   touches  pairs found;  lost  pairs the set could not place (0 unless it filled);
 *   direct   further-region weights added straight to the accumulator past a
 *            full entry buffer (not in touches; each names at most one pair);
 *   views    views counted.  NULL pointers are skipped.                     */
void scoup_uplift_touch_stats(uint64_t* touches, uint64_t* lost, uint64_t* direct, uint64_t* views);

/* Views in flight in the uplift (scoup_uplift, scoup_uplift_accumulate,
 * scoup_uplift_levels) and in scoup_render_views (whose results do not
 * depend on k at all): up to k views of a view batch are projected, binned
 * and composited at the same time, each with its own binning buffers, view i
 * on lane i mod k; lane 0 runs on the call's stream, the others on streams
 * the library creates once per device (default priority) and orders against
 * the call's stream with events.  The sum of Eq. 5 does not depend on k; the
 * deferred further-region weights of different views may reach the
 * accumulator in another order (float rounding only).  k is clamped to
 * [1, 4]; the default is 4.  The workspace sizes returned by the
 * *_workspace_bytes functions cover 4 views in flight, so k may change
 * between calls.  Process-wide setting, read at each call;
 * scoup_views_in_flight returns the current value. */
void scoup_set_views_in_flight(int32_t k);
int32_t scoup_views_in_flight(void);

/* Deferred further-region entries of the uplift: an 8x8 block whose pixels
 * fall into more regions (over all levels) than its two record regions keeps
 * the weights of the others as (Gaussian, level, region, weight) entries in a
 * per-view buffer of the workspace, added to the accumulator after the view;
 * once that buffer is full the compositing adds such weights to the
 * accumulator directly with atomics (same sums, other float rounding order).
 * scoup_set_deferred_entry_limit(n) caps the buffer at n entries per view
 * (n <= 0 restores the workspace's own capacity), so the direct path can be
 * exercised on small inputs.  Process-wide, read at each call.              */
void scoup_set_deferred_entry_limit(int64_t n);

/* ---------------------------------------------------------------------------
 * Several semantic levels in one pass (Sec. 4.1: SAM masks at three
 * granularities, each level run independently).  The blending weights e of
 * Eq. 2 do not depend on the level, so one projection / binning / compositing
 * pass per view serves every level; each level has its own region maps,
 * codes, accumulator and Top-K output.  Results equal n_levels separate
 * scoup_uplift calls.
 * ------------------------------------------------------------------------- */

/* Workspace bytes for scoup_uplift_levels (records are kept per level). */
size_t scoup_uplift_levels_workspace_bytes(int64_t n_gaussians, int32_t n_levels,
                                           const scoup_views* levels, int64_t pair_capacity,
                                           int32_t view_batch);

/* levels     host [n_levels], 1 <= n_levels <= 4; identical cameras and m_atoms,
 *            own region maps, region bases and code tables
 * k          Top-K size (0: accumulate only, no Top-K)
 * acc        host array [n_levels] of device float32 [n*m] accumulators (zeroed here)
 * topk_idx   host array [n_levels] of device int32 [n*k] (ignored if k == 0)
 * topk_val   host array [n_levels] of device float32 [n*k]
 * entropy    NULL, or host array [n_levels] of device float32 [n] (NULL entries
 *            skipped): each Gaussian's row entropy as scoup_entropy, computed
 *            from the rows while they are on chip
 * Other arguments and errors as scoup_uplift.                               */
scoup_status scoup_uplift_levels(const scoup_gaussians* g, int32_t n_levels, const scoup_views* levels,
                                 int32_t k, float* const* acc, int32_t* const* topk_idx,
                                 float* const* topk_val, float* const* entropy,
                                 int64_t pair_capacity, int32_t view_batch,
                                 void* ws, size_t ws_bytes, unsigned long long* n_contrib,
                                 void* stream);

/* Thread-local message for the last non-OK status ("" if none). */
const char* scoup_last_error(void);

/* Library version string. */
const char* scoup_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SCOUP_H_ */
