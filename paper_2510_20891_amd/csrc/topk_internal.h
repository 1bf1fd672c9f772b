// Launch interface of the top-k kernels (exact radix select over the
// statistic vector of one or many scoring problems).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "score_internal.h"

namespace emri {

constexpr int TOPK_HIST = 4096;        // bins of one radix pass (digits of at most 12 bits)
constexpr int TOPK_GATHER = 2048;      // (key, index) words the last key pass may order in LDS

// Top-k state of one job.  The histograms and counters must be zero before
// the first pass: topk_state_reset, run by the prep kernels ahead of the
// scores, clears them, and every pass leaves them so again; the other fields
// are written by the passes before they are read.
constexpr int TOPK_GROUPS = 8;           // workgroup b of a pass belongs to group b mod 8
constexpr int TOPK_ARRIVE_STRIDE = 32;   // words between arrival counters: one 128-byte line each

struct TopkState {
  uint32_t key_prefix;        // bits of the k-th largest key found so far
  uint32_t need;              // elements still to take among keys matching the prefix
  uint32_t idx_prefix;        // bits of the index threshold among tied keys
  uint32_t idx_need;
  uint32_t tie_mode;          // 1: keys equal to the threshold are cut by index
  uint32_t count;             // compaction cursor
  uint32_t eq_count;          // number of keys equal to the threshold
  uint32_t done;              // groups of the current pass that have finished
  uint32_t gathered;          // 1: the last key pass gathers and orders the winners itself
  uint32_t bcount;            // gathering cursor of the boundary words
  uint32_t fast;              // 1: the sampled pass has written the outputs (jobs with fast_r)
  uint32_t fcount;            // gathering cursor of the sampled pass
  uint32_t pad[20];
  uint32_t arrive[TOPK_GROUPS * TOPK_ARRIVE_STRIDE];   // finished workgroups of each group
  uint32_t hist[TOPK_HIST];                          // histogram of the pass, all groups
  uint32_t ghist[TOPK_GROUPS][TOPK_HIST];            // histogram of the pass, one group
};

// Part `part` of `parts` of the reset; called by every thread of a workgroup.
__device__ __forceinline__ void topk_state_reset(TopkState *st, int part, int parts) {
  constexpr int words = (int)((sizeof(TopkState) - offsetof(TopkState, arrive)) / sizeof(uint32_t));
  uint32_t *z = st->arrive;          // arrive, hist and ghist are contiguous
  const int lo = words * part / parts, hi = words * (part + 1) / parts;
  for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) z[i] = 0u;
  if (part == 0 && threadIdx.x == 0) {
    st->done = 0u;
    st->fcount = 0u;
  }
}

// One top-k problem: the statistic, its length, and where state and results live.
struct TopkJob {
  const float *stat;
  int64_t n;
  int top_k;
  uint32_t kk;                 // min(n, top_k)
  TopkState *st;
  unsigned long long *cand;    // kk candidate (key, index) pairs
  unsigned long long *bnd;     // TOPK_GATHER words: keys sharing the k-th key's 22 leading bits
  float *vals;
  int64_t *idx;
  int32_t first_block;         // this job's workgroups in a job-table launch:
  int32_t nblk;                //   first_block .. first_block + nblk - 1
  uint32_t fast_r;             // 0, or the sample rank of the sampled threshold (topk_fast_rank)
};

// A device table of jobs with the job of every workgroup (block_job), or one
// job by value (jobs == null; the whole grid works on it).
struct TopkJobs {
  const TopkJob *jobs;
  const int32_t *block_job;
  TopkJob single;
};

// Sampled threshold.  For a long statistic and a small k, two histogram
// passes over a sample (one unit of 64 consecutive statistics in every
// TOPK_SAMPLE) find the key of the sample's r-th largest element; one pass
// over the whole vector then gathers every element whose key shares or
// exceeds that key's 22 leading bits.  If at least kk and at most
// TOPK_GATHER elements were gathered, they hold the top-k (every element left
// out ranks below kk gathered ones) and are ordered in LDS; otherwise the
// radix passes run as usual.  r is chosen so that the gathered count lies
// well inside those limits unless the statistics are ordered against the
// sample.
constexpr int TOPK_SAMPLE = 16;
constexpr int TOPK_FAST_MAX_K = 256;
constexpr int64_t TOPK_FAST_MIN_N = (int64_t)1 << 16;   // jobs longer than this
// The sample rank for a job of n elements and kk = min(n, top_k) winners, or 0
// (radix passes only).
uint32_t topk_fast_rank(int64_t n, uint32_t kk);

size_t topk_workspace_bytes(int top_k);
TopkJob make_topk_job(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws);
// Workgroups per job: sets first_block and nblk of every job, returns their sum.
int64_t topk_assign_blocks(TopkJob *jobs, int n_jobs, int cu_count);
// Upper bound of topk_assign_blocks over every device, for workspace layouts.
int64_t topk_max_blocks(const int64_t *n, int n_jobs);
// fast: some job has fast_r != 0 (the sampled passes are launched first)
hipError_t launch_topk_jobs(const TopkJobs &J, int64_t total_blocks, int64_t max_n, hipStream_t stream,
                            int first_pass = 0, bool fast = false);
// first_pass = 1: the scoring launch has already run the first key pass
hipError_t launch_topk(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws, int cu_count,
                       hipStream_t stream, int first_pass = 0);

}  // namespace emri
