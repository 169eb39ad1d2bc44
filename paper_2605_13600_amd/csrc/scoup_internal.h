// Host-side launcher interface between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "scoup_device.h"

namespace scoup {

enum Stage { kStProject = 0, kStScan, kStEmit, kStSortBig, kStComposite, kStTopk, kStRender, kStDecode,
             kStRenderBwd, kStBwdGemm, kStRowBuild, kStRelevancy, kStRelPrep, kStApplyExtra, kNumStages };

// Records a HIP event pair around each launch when stage timing is enabled.
struct StageTimer {
  static bool enabled();
  static void begin(int stage, hipStream_t s);
  static void end(int stage, hipStream_t s);
  static void collect();   // after the stream is synchronised
};

// Projection + tile binning + per-tile depth order of one view.
struct BinArgs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacities;
  long long n;
  CamDev cam;
  int tile_shift;          // tile edge = 1 << tile_shift pixels
  int tiles_x, n_tiles;
  int sort_cap;            // tiles with longer lists are sorted in global memory
  GSplat* splats;          // [n]
  unsigned int* offsets;   // [n+1] Gaussian-major pair offsets (exclusive scan of tile counts)
  unsigned long long* scan_part;   // [scan blocks]
  unsigned int* tile_ids[2];       // [capacity] x 2
  unsigned long long* keys[2];     // [capacity] x 2, depth bits << 32 | gaussian id
  unsigned int* radix_hist;        // [128 * radix blocks]
  unsigned int* tile_start;        // [n_tiles + 1]
  unsigned int* big_tiles;         // [n_tiles] tiles longer than sort_cap
  unsigned int* tile_order;        // [n_tiles] tiles by descending list length (compositing order)
  float2* cull_records[4];         // uplift: per level, the view's records; pairs whose block the
  int n_cull_records;              // Gaussian cannot reach get zero records here (0 levels: none)
  unsigned int* bin_hist;          // [count_groups(n) x n_tiles] counting-pass bases, or NULL (radix path)
  long long capacity;
  Status* status;
  int sorted;              // set by launch_bin_view: which buffer holds the sorted pairs
  int pair_index;          // leave each Gaussian's first pair index in its splat (also done when
                           // n_cull_records > 0): pair (i, b) has slot offsets[i] + b's index in i's box
};

hipError_t launch_bin_view(BinArgs& a, hipStream_t s);

// Pair counts of up to kCountCams views in one pass: totals[v] += pairs of
// view v (the counts launch_bin_view's scan will find), for a capacity check
// before anything is written.
constexpr int kCountCams = 32;
struct CamBatch {
  CamDev c[kCountCams];
  int n;
};
hipError_t launch_count_view_pairs(const float* means, const float* log_scales, const float* quats,
                                   const float* opacities, long long n, const CamBatch& cams, int tile_shift,
                                   unsigned long long* totals, hipStream_t s);
int radix_passes(int n_tiles);
long long radix_blocks(long long capacity);
long long scan_blocks(long long n);
int count_groups(long long n);
hipError_t binning_set_lds_limits();
bool count_binning_ok(long long n, int n_tiles);

// One view of the uplift: composite + per-(Gaussian, block) region records,
// for up to kMaxLevels region maps (semantic levels) sharing one compositing.
constexpr int kMaxLevels = 4;
struct LevelView {
  const int* rmap;         // this view's region map of the level
  int n_regions;
  long long region_base;
  const int* code_idx;
  const float* code_val;
  int k_code;
  float* acc;              // regions beyond a block's two record slots are added here (k_apply_extra)
  float2* records;         // [2 * capacity] (global region id as int bits, weight)
  const float* dense_F;    // dense feature uplift: region features [R x dense_d] (else NULL);
  int dense_d;             //   extra regions then add w F_r to acc (N x dense_d) and w to zsum
  float* zsum;
};
struct UpliftViewArgs {
  BinArgs bin;
  int n_levels, m_atoms;
  LevelView lv[kMaxLevels];
  float4* extra;           // [extra_cap] deferred weights of regions beyond a block's two record
  unsigned int extra_cap;  //   regions: (Gaussian id, level, global region id as int bits, weight)
  int count_touches;       // statistics: count the view's distinct (Gaussian, region) pairs (level 0)
};
hipError_t launch_uplift_view(UpliftViewArgs& a, hipStream_t s);

// Sum the records of a batch of views into the accumulator rows (and Top-K).
struct RowBuildArgs {
  long long n;
  int m_atoms, k_code;
  const int* code_idx;
  const float* code_val;
  long long r_total;               // code table rows; records naming others are ignored
  int n_views;                     // views in the batch
  const unsigned int* offsets;     // [n_views][n+1]
  const float2* records;           // [n_views][2 * capacity]
  long long capacity;
  float* acc;
  int k_top;                       // 0: no Top-K
  int* topk_idx;
  float* topk_val;
  float* entropy;                  // [n] row entropy on the last pass, or NULL
  Status* status;
};
hipError_t launch_rowbuild(const RowBuildArgs& a, hipStream_t s);

// Render of one camera (Eq. 7), optionally fused with the decode (Eq. 8):
// binning, then one workgroup per 8x8 block.
struct RenderBlockArgs {
  BinArgs bin;
  const int* topk_idx;     // [n x k]
  const float* topk_val;
  int k, m_atoms;
  void* map;               // coefficient map [P x m] of map_dtype (times map_scale), or NULL
  int map_dtype;
  float map_scale;
  float* t_final;          // [P] or NULL
  int in_dtype;            // decode precision (scoup_dtype), or -1: no decode
  int out_dtype;           // features F32 / BF16
  const void* codebook_prep;   // launch_prep_codebook layout (kpad x npad)
  const float* cb_scale;   // FP8 codebook scale (device), else NULL
  int d, kpad, npad;
  float q_scale;           // FP8: coefficients are converted times this
  float out_mul;           // 1 / q_scale (FP8) or 1
  void* features;          // [P x d] of out_dtype
};
hipError_t launch_render_block(RenderBlockArgs& a, hipStream_t s, int stage);
size_t render_block_lds_bytes(const RenderBlockArgs& a);
hipError_t render_set_lds_limits();

struct DecodeArgs {
  const void* coeff;       // [P x m] in in_dtype
  long long P;
  int m, d, kpad;
  int in_dtype, out_dtype;
  const void* codebook_prep;   // codebook in MFMA B-fragment order (launch_prep_codebook)
  const float* cb_scale;       // device scale applied to the FP8 codebook (NULL otherwise)
  float out_mul;               // 1 / coefficient scale
  void* out;                   // [P x ldo] in out_dtype, columns < d written
  int ldo;                     // output row stride (0 = d)
};
int decode_kpad(int m, int in_dtype);
int decode_npad(int d);
size_t decode_codebook_bytes(int m, int d, int in_dtype);
hipError_t launch_prep_codebook(const float* C, int m, int d, int in_dtype, void* out, float* scale,
                                hipStream_t s, int transposed = 0);
hipError_t launch_decode(const DecodeArgs& a, hipStream_t s, int stage = kStDecode);

struct RelevancyArgs {
  const void* coeff;           // [P x m] coefficient map in in_dtype
  long long P;
  int m, d, in_dtype;
  const float* codebook;       // [m x d] float32
  const float* queries;        // [Q x d] float32
  const float* canon;          // [n_canon x d] float32
  int Q, n_canon;
  float temperature;
  float out_mul;               // 1 / coefficient scale
  void* frag;                  // relevancy_frag_bytes(m, Q, in_dtype) of workspace
  float* out;                  // [P x Q] float32 scores
};
int relevancy_groups(int q);
size_t relevancy_frag_bytes(int m, int q, int in_dtype);
hipError_t launch_relevancy(const RelevancyArgs& a, hipStream_t s);

constexpr int kBwdKMax = 16;        // Top-K slots the render backward supports
constexpr int kGemmMaxParts = 512;  // chunk x tile partial products of the dL/dC GEMM (<= 32 MB)
struct RenderBwdArgs {
  BinArgs bin;                 // binned (launch_bin_view) with pair_index set
  const int* topk_idx;
  const float* topk_val;
  int k, m_atoms;
  const float* dW;             // [P x m] float32 gradient of the coefficient map
  float* pair_part;            // [capacity x k] per-(Gaussian, block) partial sums (workspace)
  float* grad_val;             // [N x k] float32, accumulated
};
hipError_t launch_render_bwd_view(RenderBwdArgs& a, hipStream_t s);
hipError_t render_bwd_set_lds_limits();
// grad_C[m x d] += coeff^T [m x P] * G [P x d], float32 MFMA: per-chunk partial
// products in `part` (gemm_at_b_chunks(P, m, d) x m x d floats), then summed in
// chunk order; nothing is added when st reports a pair overflow.
int gemm_at_b_chunks(long long P, int m, int d);
hipError_t launch_gemm_at_b(const float* coeff, const float* G, long long P, int m, int d, float* part,
                            float* grad_C, const Status* st, hipStream_t s);
hipError_t decode_set_lds_limits();
hipError_t launch_topk(const float* acc, long long n, int m, int k, int* idx, float* val, hipStream_t s);
hipError_t launch_entropy(const float* acc, long long n, int m, float* out, hipStream_t s);
hipError_t launch_region_features(const int* code_idx, const float* code_val, long long r_total, int k_code,
                                  const float* C, int m, int d, float* F, Status* st, hipStream_t s);
hipError_t launch_rowbuild_dense(long long n, int d, const float* F, long long r_total, int n_views,
                                 const unsigned int* offsets, const float2* records, long long capacity,
                                 float* feat, float* zsum, int accumulate, int final_pass, hipStream_t s);
hipError_t launch_add_contrib(unsigned long long* dst, const Status* st, hipStream_t s);

}  // namespace scoup
