// Exact, deterministic top-k of the statistic vector (Sec. II D keeps the
// best-scoring candidates of a batch).  Order: decreasing S, then increasing
// template index; NaN ranks below every number and -0 equals +0.
//
// Radix select on an order-preserving 32-bit key of S: three histogram passes
// (12, 10 and 10 bits) find the key T of the k-th element and how many of the
// elements equal to T belong to the top-k.  If T is shared by more elements
// than are needed, index passes (digits of at most 12 bits over the bits an
// index of this length has) select the needed count of smallest template
// indices among them; otherwise they return at once.  One compaction pass then
// gathers exactly k (key, index) pairs and orders them.  Every pass streams
// the statistic with 16-byte loads and builds its histogram in LDS; the
// histograms of all workgroups are merged in two levels, and the last
// workgroup of a pass to finish (arrival counters in the state; no workgroup
// ever waits for another) picks the digit for the next pass or, in the
// compaction pass, orders the winners, so a top-k is 4 to 7 launches.
//
// Ahead of them, a long statistic with a small k may take the sampled
// threshold (two histogram passes over a 1/16 sample and one gathering pass;
// see topk_fast_rank), after which the radix passes of that job return at
// once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "score_internal.h"
#include "topk_internal.h"
#include "topk_device.h"

namespace emri {
namespace {

// The job of this workgroup, its index among the job's workgroups and their
// count: from the job table through block_job, or the single job passed by
// value (then the whole grid works on it).
struct JobShare {
  TopkJob job;
  int lb, nblk;
};

__device__ __forceinline__ JobShare job_of(const TopkJobs &J) {
  if (J.jobs == nullptr) return JobShare{J.single, (int)blockIdx.x, (int)gridDim.x};
  const int32_t j = load_uniform(J.block_job + blockIdx.x);
  const TopkJob job = load_uniform(J.jobs + j);
  return JobShare{job, (int)blockIdx.x - job.first_block, job.nblk};
}

// The sampled passes have written this job's outputs.
__device__ __forceinline__ bool fast_done(const TopkJob &job) { return job.fast_r != 0u && job.st->fast != 0u; }

// Outputs from sorted candidates (or none): positions past kk get -inf / -1.
__device__ __forceinline__ void write_results(const TopkJob &job, const unsigned long long *s) {
  const int kk = (int)job.kk;
  for (int i = threadIdx.x; i < job.top_k; i += blockDim.x) {
    if (i < kk) {
      const unsigned long long c = s[i];
      job.vals[i] = key_value((uint32_t)(c >> 32));
      job.idx[i] = (int64_t)(0xffffffffu - (uint32_t)(c & 0xffffffffull));
    } else {
      job.vals[i] = -__builtin_inff();
      job.idx[i] = -1;
    }
  }
}

// Bitonic network over the p2 (a power of two) words of s: decreasing order.
__device__ void sort_descending(unsigned long long *s, int p2) {
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        const int partner = i ^ stride;
        if (partner > i) {
          const bool desc = (i & size) == 0;
          const unsigned long long a = s[i], b = s[partner];
          if (desc ? (a < b) : (a > b)) {
            s[i] = b;
            s[partner] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// A word's place among nc distinct words is the number of larger words; each
// thread ranks M of them against all, and those placed below kk are written.
template <int M>
__device__ void rank_and_write(const TopkJob &job, unsigned long long *s, int nc, int cap) {
  unsigned long long w[M];
  int rank[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    w[m] = i < nc ? s[i] : ~0ull;
    rank[m] = 0;
  }
  // zero words (below every candidate) pad the list to a multiple of 8
  if (threadIdx.x < 8 && nc + (int)threadIdx.x < cap) s[nc + threadIdx.x] = 0ull;
  __syncthreads();
  const int n8 = ((nc + 7) & ~7) < cap ? ((nc + 7) & ~7) : cap;
#pragma unroll 8
  for (int j = 0; j < n8; ++j) {
    const unsigned long long o = s[j];
#pragma unroll
    for (int m = 0; m < M; ++m) rank[m] += o > w[m] ? 1 : 0;
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    if (i < nc && rank[m] < (int)job.kk) {
      job.vals[rank[m]] = key_value((uint32_t)(w[m] >> 32));
      job.idx[rank[m]] = (int64_t)(0xffffffffu - (uint32_t)(w[m] & 0xffffffffull));
    }
  }
  for (int i = (int)job.kk + threadIdx.x; i < job.top_k; i += blockDim.x) {
    job.vals[i] = -__builtin_inff();
    job.idx[i] = -1;
  }
}

// Orders the nc >= kk distinct (key, index) words in s[0..nc) (LDS, room for
// cap words) in decreasing order and writes the largest kk as the outputs;
// the whole workgroup calls it.  Up to RANK_SORT_MAX words by rank counting,
// above by a bitonic network over the next power of two.
__device__ void order_and_write(const TopkJob &job, unsigned long long *s, int nc, int cap) {
  if (nc <= HIST_THREADS) return rank_and_write<1>(job, s, nc, cap);
  if (nc <= 2 * HIST_THREADS) return rank_and_write<2>(job, s, nc, cap);
  if (nc <= 3 * HIST_THREADS) return rank_and_write<3>(job, s, nc, cap);
  if (nc <= RANK_SORT_MAX) return rank_and_write<RANK_SORT_MAX / HIST_THREADS>(job, s, nc, cap);
  int p2 = 1;
  while (p2 < nc) p2 <<= 1;
  for (int i = nc + threadIdx.x; i < p2; i += blockDim.x) s[i] = 0ull;
  __syncthreads();
  sort_descending(s, p2);
  write_results(job, s);
}

// Gathering form of the last key pass, taken when the second pass found that
// the keys sharing the k-th key's 22 leading bits (the boundary) and the kk
// winners fit in LDS together.  Keys above the boundary are winners, exactly
// kk - need of them; the boundary words are gathered too, and the last
// workgroup keeps the `need` largest of them by rank (keys, then smaller
// indices, decide: the words are distinct), then orders all kk winners.  This
// replaces the third digit pass, the index passes and the compaction pass.
__device__ void gather_winners(const JobShare &js, unsigned long long *s) {
  const TopkJob &job = js.job;
  TopkState *st = job.st;
  const uint32_t P = st->key_prefix >> 10;
  const uint32_t need = st->need, above = job.kk - need;
  for_each_stat(job.stat, job.n, js.lb, js.nblk, [&](int64_t i, float v) {
    const uint32_t k = order_key(v);
    const uint32_t hk = k >> 10;
    if (hk >= P) {
      const unsigned long long w = ((unsigned long long)k << 32) | (0xffffffffu - (uint32_t)i);
      if (hk > P) {
        const uint32_t pos = atomicAdd(&st->count, 1u);
        if (pos < above) put_candidate(job.cand + pos, w);
      } else {
        const uint32_t pos = atomicAdd(&st->bcount, 1u);
        if (pos < (uint32_t)TOPK_GATHER) put_candidate(job.bnd + pos, w);
      }
    }
  });
  if (!finish_pass<HIST_THREADS>(st, 0, js.lb, js.nblk)) return;
  if (threadIdx.x == 0) clear_bin(&st->done);
  const uint32_t nbw = read_bin(&st->bcount);
  const int nb = (int)(nbw < (uint32_t)TOPK_GATHER ? nbw : (uint32_t)TOPK_GATHER);
  constexpr int PER = TOPK_GATHER / HIST_THREADS;
  // boundary words into LDS (loads first, clamped in bounds, no branches)
  unsigned long long w[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    w[m] = get_candidate(job.bnd + (i < nb ? i : (nb > 0 ? nb - 1 : 0)));
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    if (i < nb) s[i] = w[m];
    else w[m] = 0ull;
  }
  __syncthreads();
  int rank[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) rank[m] = 0;
  for (int j = 0; j < nb; ++j) {
    const unsigned long long o = s[j];
#pragma unroll
    for (int m = 0; m < PER; ++m) rank[m] += o > w[m] ? 1 : 0;
  }
  __syncthreads();
  // winners: those above the boundary from the candidate list, then the
  // `need` largest boundary words at their ranks
  unsigned long long c[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    c[m] = get_candidate(job.cand + (i < (int)above ? i : (above > 0 ? (int)above - 1 : 0)));
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    if (i < (int)above) s[i] = c[m];
    if (i < nb && rank[m] < (int)need) s[above + rank[m]] = w[m];
  }
  __syncthreads();
  order_and_write(job, s, (int)job.kk, TOPK_GATHER);
}

// Key pass `pass` (0, 1, 2): histogram of digit [shift, shift+width) of the
// keys that match the prefix found so far.  The last pass instead gathers
// and orders the winners when the second pass found that they fit.
__global__ __launch_bounds__(HIST_THREADS) void topk_key_pass_kernel(TopkJobs J, int shift, int width, int pass) {
  const JobShare js = job_of(J);
  const TopkJob &job = js.job;
  if (job.kk == 0 || fast_done(job)) return;
  __shared__ uint32_t lh[TOPK_HIST];
  if (pass == 2 && job.st->gathered != 0u) {
    gather_winners(js, reinterpret_cast<unsigned long long *>(lh));
    return;
  }
  const int nb = 1 << width;
  clear_hist(lh, nb);
  const int hi = shift + width;
  const uint32_t prefix = pass == 0 ? 0u : job.st->key_prefix;
  const uint32_t mask = (uint32_t)nb - 1u;
  if (pass == 0) {
    first_digit_hist(job.stat, job.n, js.lb, js.nblk, lh, shift, mask);
  } else {
    for_each_stat(job.stat, job.n, js.lb, js.nblk, [&](int64_t, float v) {
      const uint32_t k = order_key(v);
      hist_add<false>(lh, (k >> shift) & mask, (k >> hi) == (prefix >> hi));
    });
  }
  flush_hist(lh, job.st->ghist[js.lb % TOPK_GROUPS], nb);
  if (finish_pass<HIST_THREADS>(job.st, nb, js.lb, js.nblk))
    select_digit<true, HIST_THREADS>(job, lh, shift, width, pass == 0, pass == 1, pass == 2);
}

// Index pass: among keys equal to the threshold, histogram of index digit
// [shift, shift+width) of the indices that match the index prefix so far.
__global__ __launch_bounds__(HIST_THREADS) void topk_index_pass_kernel(TopkJobs J, int shift, int width, int first) {
  const JobShare js = job_of(J);
  const TopkJob &job = js.job;
  if (job.kk == 0 || fast_done(job) || job.st->tie_mode == 0u) return;
  __shared__ uint32_t lh[TOPK_HIST];
  const int nb = 1 << width;
  clear_hist(lh, nb);
  const int hi = shift + width;
  const uint32_t key = job.st->key_prefix;
  const uint32_t prefix = first ? 0u : job.st->idx_prefix;
  const uint32_t mask = (uint32_t)nb - 1u;
  for_each_stat(job.stat, job.n, js.lb, js.nblk, [&](int64_t i, float v) {
    const uint32_t u = (uint32_t)i;
    hist_add<true>(lh, (u >> shift) & mask, order_key(v) == key && (hi >= 32 || (u >> hi) == (prefix >> hi)));
  });
  flush_hist(lh, job.st->ghist[js.lb % TOPK_GROUPS], nb);
  if (finish_pass<HIST_THREADS>(job.st, nb, js.lb, js.nblk))
    select_digit<false, HIST_THREADS>(job, lh, shift, width, first != 0, false, false);
}

// Compaction: every element above the threshold, and those equal to it that
// are needed (all, or those with index <= the index threshold), go to the
// candidate list; the last workgroup sorts the kk candidates (descending key,
// then ascending index, both encoded in one 64-bit word) and writes the outputs.
__global__ __launch_bounds__(HIST_THREADS) void topk_compact_kernel(TopkJobs J) {
  const JobShare js = job_of(J);
  const TopkJob &job = js.job;
  __shared__ unsigned long long s[EMRI_MAX_TOPK];
  if (job.kk == 0) {
    if (js.lb == 0) write_results(job, s);
    return;
  }
  if (fast_done(job)) return;                     // the sampled passes have done it
  TopkState *st = job.st;
  if (st->gathered != 0u) return;                 // the last key pass has done it
  const uint32_t key = st->key_prefix;
  const bool tie = st->tie_mode != 0u;
  const uint32_t thr = st->idx_prefix;
  const uint32_t kk = job.kk;
  unsigned long long *cand = job.cand;
  for_each_stat(job.stat, job.n, js.lb, js.nblk, [&](int64_t i, float v) {
    const uint32_t k = order_key(v);
    const bool sel = k > key || (k == key && (!tie || (uint32_t)i <= thr));
    if (sel) {
      const uint32_t pos = atomicAdd(&st->count, 1u);
      if (pos < kk) put_candidate(cand + pos, ((unsigned long long)k << 32) | (0xffffffffu - (uint32_t)i));
    }
  });
  if (!finish_pass<HIST_THREADS>(st, 0, js.lb, js.nblk)) return;
  if (threadIdx.x == 0) clear_bin(&st->done);
  const int nc = (int)kk;
  {
    constexpr int PER = EMRI_MAX_TOPK / HIST_THREADS;
    unsigned long long c[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int i = threadIdx.x + m * HIST_THREADS;
      c[m] = get_candidate(cand + (i < nc ? i : nc - 1));        // in bounds, no branch
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int i = threadIdx.x + m * HIST_THREADS;
      if (i < nc) s[i] = c[m];
    }
  }
  __syncthreads();
  order_and_write(job, s, nc, EMRI_MAX_TOPK);
}


// Calls f(stat[i]) for this workgroup's share of the sample: unit u of 64
// statistics (16 groups of 4) is sampled when u is a multiple of TOPK_SAMPLE;
// the statistics past the last whole group of 4 are not sampled.
template <typename F>
__device__ __forceinline__ void for_each_sample(const float *__restrict__ stat, int64_t n, int lb, int nblk, F &&f) {
  const int64_t n4 = n >> 2;
  const int64_t slots = (n4 + 16 * TOPK_SAMPLE - 1) / (16 * TOPK_SAMPLE) * 16;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const gmem<const f4> *s4 = global(reinterpret_cast<const f4 *>(stat));
  for (int64_t s0 = (int64_t)lb * blockDim.x + threadIdx.x; s0 < slots; s0 += STREAM * stride) {
    f4 v[STREAM];
    bool live[STREAM];
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      const int64_t sl = s0 + u * stride;
      const int64_t q = (sl >> 4) * (16 * TOPK_SAMPLE) + (sl & 15);
      live[u] = sl < slots && q < n4;
      v[u] = live[u] ? s4[q] : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      if (live[u]) {
        f(v[u].x);
        f(v[u].y);
        f(v[u].z);
        f(v[u].w);
      }
    }
  }
}

// Sampled pass `pass` (0, 1): histogram of key digit [shift, shift+width) of
// the sampled keys that match the prefix so far; the last workgroup fixes
// the digit of the sample's fast_r-th largest key (22 leading bits after the
// second pass).
__global__ __launch_bounds__(HIST_THREADS) void topk_sample_pass_kernel(TopkJobs J, int shift, int width, int pass) {
  const JobShare js = job_of(J);
  const TopkJob &job = js.job;
  if (job.fast_r == 0u) return;
  __shared__ uint32_t lh[TOPK_HIST];
  const int nb = 1 << width;
  clear_hist(lh, nb);
  const int hi = shift + width;
  const uint32_t prefix = pass == 0 ? 0u : job.st->key_prefix;
  const uint32_t mask = (uint32_t)nb - 1u;
  if (pass == 0) {
    for_each_sample(job.stat, job.n, js.lb, js.nblk,
                    [&](float v) { hist_add<true>(lh, (order_key(v) >> shift) & mask, true); });
  } else {
    for_each_sample(job.stat, job.n, js.lb, js.nblk, [&](float v) {
      const uint32_t k = order_key(v);
      hist_add<false>(lh, (k >> shift) & mask, (k >> hi) == (prefix >> hi));
    });
  }
  flush_hist(lh, job.st->ghist[js.lb % TOPK_GROUPS], nb);
  if (finish_pass<HIST_THREADS>(job.st, nb, js.lb, js.nblk))
    select_digit<true, HIST_THREADS>(job, lh, shift, width, pass == 0, false, false, job.fast_r);
}

// Gathering pass of the sampled threshold: every element whose key's 22
// leading bits are at least those of the sample's fast_r-th largest key is
// a candidate.  A workgroup collects its candidates in LDS and moves them to
// the boundary list with one global atomic; a workgroup with more than
// TOPK_GATHER of them makes the job's count exceed TOPK_GATHER.  The last
// workgroup checks that kk to TOPK_GATHER candidates were gathered; then it
// orders them and writes the outputs (and the radix passes return at once),
// else it leaves the job to the radix passes.
__global__ __launch_bounds__(HIST_THREADS) void topk_fast_gather_kernel(TopkJobs J) {
  const JobShare js = job_of(J);
  const TopkJob &job = js.job;
  if (job.fast_r == 0u) return;
  __shared__ unsigned long long s[TOPK_GATHER];
  __shared__ uint32_t n_local, base, n_ok;
  TopkState *st = job.st;
  const uint32_t P = st->key_prefix >> 10;
  if (threadIdx.x == 0) n_local = 0u;
  __syncthreads();
  const auto take = [&](int64_t i, float v) {
    const uint32_t k = order_key(v);
    if ((k >> 10) >= P) {
      const uint32_t pos = atomicAdd(&n_local, 1u);
      if (pos < (uint32_t)TOPK_GATHER) s[pos] = ((unsigned long long)k << 32) | (0xffffffffu - (uint32_t)i);
    }
  };
  // Keys of at least T = P << 10 are candidates.  When T is a non-negative
  // number's key, that is v >= key_value(T) in FP32 (NaN compares false, -0
  // equals +0), so a group of loads without a candidate costs one compare per
  // element and the keys are formed only for groups that hold one.
  const uint32_t T = P << 10;
  const bool pos_thr = T >= 0x80000000u;
  const float tf = key_value(T);
  typedef float f4 __attribute__((ext_vector_type(4)));
  const gmem<const f4> *s4 = global(reinterpret_cast<const f4 *>(job.stat));
  const int64_t n4 = job.n >> 2;
  const int64_t stride = (int64_t)js.nblk * blockDim.x;
  for (int64_t q0 = (int64_t)js.lb * blockDim.x + threadIdx.x; q0 < n4; q0 += STREAM * stride) {
    f4 v[STREAM];
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      const int64_t q = q0 + u * stride;
      v[u] = q < n4 ? s4[q] : f4{0.f, 0.f, 0.f, 0.f};
    }
    bool any = !pos_thr;
#pragma unroll
    for (int u = 0; u < STREAM; ++u)
      any = any || v[u].x >= tf || v[u].y >= tf || v[u].z >= tf || v[u].w >= tf;
    if (any) {
#pragma unroll
      for (int u = 0; u < STREAM; ++u) {
        const int64_t q = q0 + u * stride;
        if (q < n4) {
          take(4 * q + 0, v[u].x);
          take(4 * q + 1, v[u].y);
          take(4 * q + 2, v[u].z);
          take(4 * q + 3, v[u].w);
        }
      }
    }
  }
  for (int64_t i = 4 * n4 + (int64_t)js.lb * blockDim.x + threadIdx.x; i < job.n; i += stride) take(i, job.stat[i]);
  __syncthreads();
  const uint32_t nl = n_local;
  if (threadIdx.x == 0 && nl > 0u)
    base = atomicAdd(&st->fcount, nl <= (uint32_t)TOPK_GATHER ? nl : (uint32_t)TOPK_GATHER + 1u);
  __syncthreads();
  if (nl <= (uint32_t)TOPK_GATHER) {
    for (uint32_t j = threadIdx.x; j < nl; j += HIST_THREADS)
      if (base + j < (uint32_t)TOPK_GATHER) put_candidate(job.bnd + base + j, s[j]);
  }
  if (!finish_pass<HIST_THREADS>(st, 0, js.lb, js.nblk)) return;
  if (threadIdx.x == 0) {
    clear_bin(&st->done);
    const uint32_t c = read_bin(&st->fcount);
    clear_bin(&st->fcount);
    const bool ok = c >= job.kk && c <= (uint32_t)TOPK_GATHER;
    st->fast = ok ? 1u : 0u;
    n_ok = ok ? c : 0u;
  }
  __syncthreads();
  const int nc = (int)n_ok;
  if (nc == 0) return;
  constexpr int PER = TOPK_GATHER / HIST_THREADS;
  unsigned long long w[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    w[m] = get_candidate(job.bnd + (i < nc ? i : nc - 1));        // in bounds, no branch
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int i = threadIdx.x + m * HIST_THREADS;
    if (i < nc) s[i] = w[m];
  }
  __syncthreads();
  order_and_write(job, s, nc, TOPK_GATHER);
}

}  // namespace

size_t topk_workspace_bytes(int top_k) {
  return round_up(sizeof(TopkState), 256) + round_up((size_t)(top_k > 0 ? top_k : 1) * 8, 256) +
         (size_t)TOPK_GATHER * 8;
}

TopkJob make_topk_job(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws) {
  TopkJob job;
  job.stat = stat;
  job.n = n;
  job.top_k = top_k;
  job.kk = (uint32_t)(n < (int64_t)top_k ? n : (int64_t)top_k);
  job.st = reinterpret_cast<TopkState *>(ws);
  job.cand = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) + round_up(sizeof(TopkState), 256));
  job.bnd = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) + round_up(sizeof(TopkState), 256) +
                                                   round_up((size_t)(top_k > 0 ? top_k : 1) * 8, 256));
  job.vals = vals;
  job.idx = idx;
  job.first_block = 0;
  job.nblk = 1;
  job.fast_r = 0u;
  return job;
}

// The sample holds about n/16 elements, in whole units of 64; its r-th
// largest key is expected near rank 16 r of the whole vector, i.e. about
// 2 kk + 128, with a spread of about 16 sqrt(r): the gathered count exceeds
// kk (the sample would need r of the top kk elements, about 6 standard
// deviations above the mean of kk/16 at kk = 256) and stays below
// TOPK_GATHER, unless the statistics are ordered against the sample (then the
// radix passes run).
uint32_t topk_fast_rank(int64_t n, uint32_t kk) {
  if (kk == 0u || kk > (uint32_t)TOPK_FAST_MAX_K || n <= TOPK_FAST_MIN_N) return 0u;
  return (2u * kk + TOPK_SAMPLE - 1u) / TOPK_SAMPLE + 8u;
}

namespace {
constexpr int64_t kMinShare = 4 * STREAM * HIST_THREADS;   // one group of loads per thread
constexpr int64_t kMaxBlocksPerJob = 1024;

int64_t blocks_for(int64_t n, int64_t chunk, int64_t cap) {
  return std::max<int64_t>(1, std::min(cap, (n + chunk - 1) / chunk));
}
}  // namespace

// Every workgroup takes at least one group of loads per thread; with many or
// long jobs the share grows so that all jobs together use about eight
// workgroups per CU, split in proportion to their lengths (each workgroup pays
// a fixed merge and arrival, and a job with too few workgroups streams its
// statistic at the pace of their loads in flight).  A job takes at most four
// per CU and at most 1024.
int64_t topk_assign_blocks(TopkJob *jobs, int n_jobs, int cu_count) {
  int64_t total_n = 0;
  for (int j = 0; j < n_jobs; ++j) total_n += jobs[j].n;
  // at most eight workgroups per CU in all (all resident at once), also after
  // each job rounds its share up: chunks of total / (target - jobs) elements
  const int64_t target = (int64_t)cu_count * 8;
  const int64_t parts = std::max<int64_t>(target - n_jobs, target / 2);
  const int64_t chunk = std::max<int64_t>(kMinShare, (total_n + parts - 1) / parts);
  const int64_t cap = std::min<int64_t>(kMaxBlocksPerJob, (int64_t)cu_count * 4);
  int64_t first = 0;
  for (int j = 0; j < n_jobs; ++j) {
    jobs[j].first_block = (int32_t)first;
    jobs[j].nblk = (int32_t)blocks_for(jobs[j].n, chunk, cap);
    first += jobs[j].nblk;
  }
  return first;
}

int64_t topk_max_blocks(const int64_t *n, int n_jobs) {
  int64_t total = 0;
  for (int j = 0; j < n_jobs; ++j) total += blocks_for(n[j], kMinShare, kMaxBlocksPerJob);
  return total;
}

hipError_t launch_topk_jobs(const TopkJobs &J, int64_t total_blocks, int64_t max_n, hipStream_t stream,
                            int first_pass, bool fast) {
  if (total_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_blocks), block(HIST_THREADS);
  if (fast) {
    hipLaunchKernelGGL(topk_sample_pass_kernel, grid, block, 0, stream, J, 20, 12, 0);
    hipLaunchKernelGGL(topk_sample_pass_kernel, grid, block, 0, stream, J, 10, 10, 1);
    hipLaunchKernelGGL(topk_fast_gather_kernel, grid, block, 0, stream, J);
  }
  static const int key_shift[3] = {20, 10, 0}, key_width[3] = {12, 10, 10};
  for (int pass = first_pass; pass < 3; ++pass)
    hipLaunchKernelGGL(topk_key_pass_kernel, grid, block, 0, stream, J, key_shift[pass], key_width[pass], pass);
  // index digits cover the bits of the largest index, top digit first
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < max_n) ++bits;
  for (int hi = bits; hi > 0; hi -= INDEX_DIGIT) {
    const int width = hi < INDEX_DIGIT ? hi : INDEX_DIGIT;
    hipLaunchKernelGGL(topk_index_pass_kernel, grid, block, 0, stream, J, hi - width, width, hi == bits ? 1 : 0);
  }
  hipLaunchKernelGGL(topk_compact_kernel, grid, block, 0, stream, J);
  return hipGetLastError();
}

hipError_t launch_topk(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws, int cu_count,
                       hipStream_t stream, int first_pass) {
  if (top_k <= 0) return hipSuccess;
  TopkJobs J;
  J.jobs = nullptr;
  J.block_job = nullptr;
  J.single = make_topk_job(stat, n, top_k, vals, idx, ws);
  if (first_pass == 0) J.single.fast_r = topk_fast_rank(n, J.single.kk);
  const int64_t blocks = topk_assign_blocks(&J.single, 1, cu_count);
  return launch_topk_jobs(J, blocks, n, stream, first_pass, J.single.fast_r != 0u);
}

}  // namespace emri
