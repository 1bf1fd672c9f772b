// Launch interface of the re-scoring kernels (rescore.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "score_internal.h"

namespace emri {

constexpr int RESCORE_MAX_CAND = 4096;   // candidates re-scored per call

struct RescoreParams {
  const void *power;          // spectrogram rows (FP32 or FP16)
  const double *seg;          // per segment: f0*T then U[alpha, k]*T, seg_stride doubles apart
  const float *coeffs;        // n_tmpl x K
  float *stat;                // n_tmpl: the candidates' entries are overwritten
  const int64_t *cand_idx;    // n_cand template indices
  float *cand_val;            // n_cand re-scored statistics
  int64_t n_tmpl;
  int n_cand, n_seg, seg_stride, K, row_pitch, k_min, k_max, pad;
};

// Candidates re-scored for a top_k of n_tmpl templates: min(n, max(4 top_k, 64), 4096).
int rescore_candidates(int top_k, int64_t n_tmpl);
hipError_t launch_rescore(const RescoreParams &r, int dtype, hipStream_t stream);
// Top-k of the re-scored candidates by (-S, index), padded with (-inf, -1).
hipError_t launch_rescore_select(const float *cand_val, const int64_t *cand_idx, int n_cand, int top_k,
                                 float *out_val, int64_t *out_idx, hipStream_t stream);

}  // namespace emri
