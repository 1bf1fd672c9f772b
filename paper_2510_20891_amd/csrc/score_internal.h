// Launch interface between the C ABI layer and the scoring / top-k kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "staging_geom.h"

namespace emri {

constexpr int EMRI_MAX_K = 32;
constexpr int EMRI_MAX_TOPK = 4096;

struct TopkState;

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
  int pitch_bytes;            // bytes between rows, in HBM and between LDS row buffers
  int G;                      // rows per staging step (1, 2 or 4)
  int half_bytes;             // bytes of one LDS half: lead-in + G rows rounded up to 1 KB
  uint64_t slot_owner;        // byte j: wave that re-zeroes zero slot j after a copy (0xff: none)
  // mixed-precision form only (null otherwise)
  const void *mtab;           // per segment: 3 BF16 pieces of U*T, MIXED_GROUPS(K) groups of 4 k
  const void *mseg;           // per segment: MixedSeg
  int mtab_bytes;             // bytes of mtab for round_up(n_seg, 4) segments (staged in LDS first)
  float one;                  // 1.0f: FP16 power is added as fma(P, one, acc), one instruction
  unsigned *redo;             // above K = 8: the reduced-chain launch's queue of tiles for the
                              // full chains (MIXED_REDO_BYTES; count cleared by the prep kernel), or null
  // standalone plain launches with a top-k: the top-k state whose first key
  // pass the scoring workgroups run over their own statistics, or null
  TopkState *topk;
  uint32_t topk_kk;           // min(n_tmpl, top_k)
  uint32_t redo_tag;          // recorded with each queued tile: the problem of a batched launch (0 otherwise)
};

// Mixed-precision form: per-segment offset f0*T = I + phi with I the even
// integer nearest f0*T (FP64) and phi in [-1, 1] (FP32); M = 1.5*2^23 + I in
// FP32 (exact for |I| < 2^22; segments farther out only occur for templates
// that take the FP64 path, and M is then unused).
struct MixedSeg {
  double I;
  float phi;
  float M;
};

constexpr int MIXED_MAX_K = 16;
// Queue of tiles the reduced-chain mixed launch leaves to the full chains:
// word 0 counts the entries claimed; entry e, four 32-bit words (first
// template, end of the tile, the queueing launch's redo_tag, unused), starts
// at byte 16 + 16e.  A count above the capacity sends the whole batch to the
// full chains.
constexpr int MIXED_REDO_CAP = 1024;
constexpr size_t MIXED_REDO_BYTES = 16 + 16 * (size_t)MIXED_REDO_CAP;
// Workgroup size of the mixed kernel: 1024 threads (four waves per SIMD, 128
// VGPRs each) up to K = 8, 768 (three waves, 168 VGPRs) above; the first
// SCORE_WAVES of its waves stage the rows.
__host__ __device__ constexpr int mixed_threads(int K) { return K <= 8 ? 1024 : 768; }
static_assert(mixed_threads(1) >= SCORE_THREADS && mixed_threads(16) >= SCORE_THREADS && mixed_threads(16) % 64 == 0,
              "the staging waves are a prefix of the workgroup");
__host__ __device__ constexpr int mixed_groups(int K) { return (K + 3) / 4; }
// bytes of the BF16 piece table per segment: 3 pieces x groups x 4 values x 2 bytes
__host__ __device__ constexpr int mixed_row_bytes(int K) { return 3 * mixed_groups(K) * 8; }

// LDS staging of spectrogram rows: see staging_geom.h (Staging, make_staging).

// A range of one stream's templates, scored by one workgroup of the batched
// launch.  Workgroups claim items in table order through an atomic counter.
struct BatchItem {
  int32_t stream;
  int32_t pad;
  int64_t begin, end;
};

// Everything the per-segment constants kernel needs for one stream.
struct TopkState;

struct PrepJob {
  const double *f0, *U;
  double *seg, *bound;
  unsigned long long *near_tie;
  double t_sft;
  int K, n_seg, seg_stride, pad;
  void *mtab;                  // mixed-precision tables, or null
  void *mseg;
  TopkState *topk;             // top-k state to reset, or null
  unsigned *redo;              // tile queue of the reduced-chain mixed launch (count to clear), or null
};

// Launch shape of a batched scoring launch (device tables live in the workspace).
struct BatchLaunch {
  const ScoreParams *params;
  const BatchItem *items;
  int *counter;               // next item to claim, [0] and [1] (reset to 0 by the prep kernel of each run)
  int n_items, grid, K, dtype, tpl;
  int mixed;
  size_t lds;
  unsigned *redo;             // mixed above K = 8: the tile queue of the reduced-chain launch, or null
};

// Read a small trivially copyable struct from read-only device memory with
// scalar (constant address space) loads, one dword at a time.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *src) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
  typedef const __attribute__((address_space(4))) uint32_t *cwords;
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = ((cwords)src)[i];
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

int score_templates_per_lane(int K, bool alt);
hipError_t launch_score_prep(const PrepJob &job, hipStream_t stream);
hipError_t launch_score_prep_batched(const PrepJob *jobs, int n_jobs, int *counter, hipStream_t stream);
hipError_t launch_score(const ScoreParams &p, int K, int dtype, bool validate, int grid, size_t lds,
                        hipStream_t stream);
hipError_t launch_score_batched(const BatchLaunch &b, hipStream_t stream);
// mixed-precision form (BF16-split MFMA contraction, FP64 offset and rounding)
int mixed_templates_per_lane(int K);
int mixed_tile_templates(int K);     // templates per tile of the mixed kernel
hipError_t launch_score_mixed(const ScoreParams &p, int K, int dtype, int grid, size_t lds, hipStream_t stream);
hipError_t launch_score_mixed_batched(const BatchLaunch &b, hipStream_t stream);
// multi-harmonic form (harmonics.hip): 1 <= K <= HARMONICS_MAX_K, 1 <= n_harm <= 4
constexpr int HARMONICS_MAX_K = 16;
constexpr int HARMONICS_MAX_H = 4;
hipError_t launch_score_harmonics(const ScoreParams &p, int K, int dtype, int n_harm, const double *ratios, int grid,
                                  size_t lds, hipStream_t stream);

}  // namespace emri
