// Launch interface between the C ABI layer and the scoring / top-k kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace emri {

constexpr int SCORE_THREADS = 512;   // one persistent workgroup of 8 waves per CU
constexpr int EMRI_MAX_K = 32;
constexpr int EMRI_MAX_TOPK = 4096;
constexpr int TOPK_HIST = 2048;
constexpr int SCORE_LDS_LEAD = 16;   // bytes ahead of bin 0 in each LDS row buffer

struct ScoreParams {
  const void *power;          // spectrogram rows (FP32 or FP16)
  const double *seg;          // per segment: f0*T then U[alpha, k]*T, seg_stride doubles apart
  const double *bound;        // max |f0*T|, then max_alpha |U[alpha,k]*T|
  const float *coeffs;        // n_tmpl x K
  float *stat;                // n_tmpl
  int32_t *bins;              // validation only: n_tmpl x n_seg, or null
  unsigned long long *near_tie;  // validation only, or null
  int64_t n_tmpl;
  int64_t per_block;          // templates owned by each workgroup
  int n_seg;
  int seg_stride;
  int k_min, k_max;
  int row_bytes_pitch;        // bytes between spectrogram rows
  int copy_bytes;             // bytes of a row copied to LDS (n_bins elements, 16-byte multiple)
  int row_chunks;             // 1 KB wave copies per row
  int buf_bytes;              // bytes per LDS row buffer (multiple of 16)
  int nbuf;                   // LDS row buffers: 2, 4 or 8 (two halves of G = nbuf/2 rows)
  int lo_owner, hi_owner;     // wave that re-zeroes the slot below / above the bin range after a copy (-1: none)
};

int score_templates_per_tile(int K);
hipError_t launch_score_prep(const double *f0, const double *U, int K, int n_seg, double t_sft, double scale,
                             double *seg, int seg_stride, double *bound, unsigned long long *near_tie,
                             hipStream_t stream);
hipError_t launch_score(const ScoreParams &p, int K, int dtype, bool validate, int grid, size_t lds,
                        hipStream_t stream);

struct TopkState {
  uint32_t key_prefix;        // bits of the k-th largest key found so far
  uint32_t need;              // elements still to take among keys matching the prefix
  uint32_t idx_prefix;        // bits of the index threshold among tied keys
  uint32_t idx_need;
  uint32_t tie_mode;          // 1: keys equal to the threshold are cut by index
  uint32_t count;             // compaction cursor
  uint32_t eq_count;          // number of keys equal to the threshold
  uint32_t pad;
  uint32_t hist[TOPK_HIST];
};

size_t topk_workspace_bytes(int top_k);
hipError_t launch_topk(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws, int cu_count,
                       hipStream_t stream);

}  // namespace emri
