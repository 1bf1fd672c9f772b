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
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "score_internal.h"
#include "topk_internal.h"

namespace emri {
namespace {

constexpr int HIST_THREADS = 256;

// Device-memory views: loads and stores through them are global (not flat)
// instructions, so the compiler need not order them against LDS accesses.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ gmem<T> *global(T *p) {
  return (gmem<T> *)p;
}
constexpr int INDEX_DIGIT = 12;               // widest index digit (TOPK_HIST bins)
constexpr int RANK_SORT_MAX = 1024;           // up to this many winners are ordered by rank counting

__device__ __forceinline__ uint32_t order_key(float v) {
  uint32_t u = __float_as_uint(v);
  if (v != v) return 0u;                       // NaN: lowest
  if (u == 0x80000000u) u = 0u;                // -0 -> +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Calls f(i, stat[i]) for this workgroup's share of the statistic.  Each
// thread keeps STREAM 16-byte loads in flight (a pass is one short stream over
// the vector, so latency, not bandwidth, sets its time otherwise).
constexpr int STREAM = 4;

template <typename F>
__device__ __forceinline__ void for_each_stat(const float *__restrict__ stat, int64_t n, int lb, int nblk, F &&f) {
  const int64_t n4 = n >> 2;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const gmem<const f4> *s4 = global(reinterpret_cast<const f4 *>(stat));
  for (int64_t q0 = (int64_t)lb * blockDim.x + threadIdx.x; q0 < n4; q0 += STREAM * stride) {
    f4 v[STREAM];
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      const int64_t q = q0 + u * stride;
      v[u] = q < n4 ? s4[q] : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      const int64_t q = q0 + u * stride;
      if (q < n4) {
        f(4 * q + 0, v[u].x);
        f(4 * q + 1, v[u].y);
        f(4 * q + 2, v[u].z);
        f(4 * q + 3, v[u].w);
      }
    }
  }
  for (int64_t i = 4 * n4 + (int64_t)lb * blockDim.x + threadIdx.x; i < n; i += stride) f(i, stat[i]);
}

// Count `bin` in the LDS histogram if `in`.  Statistics crowd into a few bins
// of the leading digit (and tied keys into runs of neighbouring indices), so
// with AGGREGATE the lanes of a wave that share the bin of the first lane still
// counting add their count with one atomic; after three such rounds the rest
// add one each.  Later key digits spread over their bins and count directly.
template <bool AGGREGATE>
__device__ __forceinline__ void hist_add(uint32_t *lh, uint32_t bin, bool in) {
  if (!in) return;
  for (int round = 0; round < (AGGREGATE ? 3 : 0); ++round) {
    const uint32_t lb = __builtin_amdgcn_readfirstlane(bin);     // first lane still counting
    const unsigned long long group = __ballot(bin == lb);
    if (bin == lb) {
      if (__lane_id() == __ffsll(group) - 1) atomicAdd(&lh[lb], (uint32_t)__popcll(group));
      return;
    }
  }
  atomicAdd(&lh[bin], 1u);
}

// Histogram of the first key digit (sign, exponent and three mantissa bits).
// Across a statistic vector it takes a few neighbouring values, so an LDS
// atomic per element would serialise on them.  Each thread counts the 8 bins
// of its wave's window (starting 3 below the bin of the wave's first element)
// in 8-bit fields of one 64-bit register, without branches; a group of loads
// with an element outside the window counts those elements one by one.  After
// at most 15 groups (240 elements per field) and at the end, the wave adds the
// fields up (16 bits each: at most 64 x 240 per bin) and one lane adds the 8
// sums to the LDS histogram.  Every lane of a wave runs the same number of
// groups (those the wave's first lane runs), so the wave-wide sums see all 64
// lanes; lanes past the end load the last element again and count nothing.
__device__ __forceinline__ void add_window(uint32_t *lh, uint32_t base, uint64_t packed) {
  unsigned long long even = packed & 0x00ff00ff00ff00ffull;          // bins base+0, +2, +4, +6
  unsigned long long odd = (packed >> 8) & 0x00ff00ff00ff00ffull;    // bins base+1, +3, +5, +7
  for (int off = 32; off > 0; off >>= 1) {
    even += __shfl_xor(even, off, 64);
    odd += __shfl_xor(odd, off, 64);
  }
  if (__lane_id() == 0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const uint32_t ce = (uint32_t)(even >> (16 * f)) & 0xffffu, co = (uint32_t)(odd >> (16 * f)) & 0xffffu;
      if (ce) atomicAdd(&lh[base + 2 * f], ce);
      if (co) atomicAdd(&lh[base + 2 * f + 1], co);
    }
  }
}

__device__ __forceinline__ void first_digit_hist(const float *stat, int64_t n, int lb, int nblk, uint32_t *lh, int shift,
                                                 uint32_t mask) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const gmem<const f4> *s4 = global(reinterpret_cast<const f4 *>(stat));
  const int64_t n4 = n >> 2;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  const int lane = (int)__lane_id();
  uint32_t base = 0u;
  uint64_t packed = 0ull;
  int groups = 0;
  for (int64_t q0 = (int64_t)lb * blockDim.x + threadIdx.x; q0 - lane < n4; q0 += STREAM * stride) {
    f4 v[STREAM];
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      const int64_t q = q0 + u * stride;
      v[u] = s4[q < n4 ? q : n4 - 1];
    }
    if (groups == 0) {                // the wave's first lane has an element here
      const uint32_t b0 = __builtin_amdgcn_readfirstlane((order_key(v[0].x) >> shift) & mask);
      base = b0 >= 3u ? b0 - 3u : 0u;
    }
    bool miss = false;
#pragma unroll
    for (int u = 0; u < STREAM; ++u) {
      const bool live = q0 + u * stride < n4;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t d = ((order_key(v[u][c]) >> shift) & mask) - base;
        packed += (live && d < 8u) ? 1ull << (8u * d) : 0ull;
        miss |= live && d >= 8u;
      }
    }
    if (miss) {
#pragma unroll
      for (int u = 0; u < STREAM; ++u) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t bin = (order_key(v[u][c]) >> shift) & mask;
          if (q0 + u * stride < n4 && bin - base >= 8u) atomicAdd(&lh[bin], 1u);
        }
      }
    }
    if (++groups % 15 == 0) {
      add_window(lh, base, packed);
      packed = 0ull;
    }
  }
  if (groups % 15 != 0) add_window(lh, base, packed);
  for (int64_t i = 4 * n4 + (int64_t)lb * blockDim.x + threadIdx.x; i < n; i += stride)
    atomicAdd(&lh[(order_key(stat[i]) >> shift) & mask], 1u);
}

__device__ __forceinline__ void clear_hist(uint32_t *lh, int nb) {
  for (int b = threadIdx.x; b < nb; b += blockDim.x) lh[b] = 0u;
  __syncthreads();
}

// A group histogram keeps bin b at word (b mod 8) * (TOPK_HIST / 8) + b / 8,
// so neighbouring bins, which the leading digit fills at once, sit on
// different cache lines and their atomics are not serialised together.
constexpr int GH_ROWS = 8, GH_COLS = TOPK_HIST / GH_ROWS;
// Agent-scope add to a device-memory bin (a global, not flat, atomic).
__device__ __forceinline__ void add_bin(uint32_t *bin, uint32_t v) {
  __hip_atomic_fetch_add(global(bin), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int gh_word(int b) { return (b % GH_ROWS) * GH_COLS + b / GH_ROWS; }
__device__ __forceinline__ int gh_bin(int w) { return (w % GH_COLS) * GH_ROWS + w / GH_COLS; }

__device__ __forceinline__ void flush_hist(const uint32_t *lh, uint32_t *gh, int nb) {
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    if (lh[b]) add_bin(&gh[gh_word(b)], lh[b]);
}

// Everything one workgroup leaves for another goes through agent-scope
// atomics, which are coherent across the chip's L2 caches without cache
// maintenance: histogram bins and counters by read-modify-write, merged bins
// and candidates by atomic loads and stores.  A pass merges in two levels, so
// that no address takes more than about 128 atomics (atomics on one address
// are serialised, and the workgroups of a pass finish at about the same time):
// a workgroup adds its LDS histogram into its group's histogram, waits until
// its atomics have completed (s_waitcnt) and counts itself on the group's arrival
// counter; the last of a group moves the group histogram into the pass
// histogram, waits, and counts the group on `done`; the workgroup that
// completes `done` sees every other workgroup's completed atomics.  No
// workgroup waits for another, and no pass writes back or invalidates an L2
// cache (an agent-scope fence would, once per workgroup).
__device__ __forceinline__ uint32_t read_bin(const uint32_t *bin);
__device__ __forceinline__ void clear_bin(uint32_t *bin);

__device__ __forceinline__ bool finish_pass(TopkState *st, int nb, int lb, int nblk) {
  __shared__ uint32_t flag;
  const uint32_t G = TOPK_GROUPS, g = (uint32_t)lb % G, nw = (uint32_t)nblk;
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t members = (nw - g + G - 1) / G;     // workgroups b < nblk with b mod G == g
    flag = atomicAdd(&st->arrive[g * TOPK_ARRIVE_STRIDE], 1u) == members - 1u ? 1u : 0u;
  }
  __syncthreads();
  if (flag == 0u) return false;
  if (nb > 0) {
    // all loads first (no branches between them), then the adds and clears
    constexpr int PER = TOPK_HIST / HIST_THREADS;
    uint32_t h[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) h[m] = read_bin(&st->ghist[g][threadIdx.x + m * HIST_THREADS]);
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int w = threadIdx.x + m * HIST_THREADS;
      if (h[m]) {
        add_bin(&st->hist[gh_bin(w)], h[m]);
        clear_bin(&st->ghist[g][w]);
      }
    }
  }
  if (threadIdx.x == 0) clear_bin(&st->arrive[g * TOPK_ARRIVE_STRIDE]);
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t groups = nw < G ? nw : G;
    flag = atomicAdd(&st->done, 1u) == groups - 1u ? 1u : 0u;
  }
  __syncthreads();
  return flag != 0u;
}

__device__ __forceinline__ uint32_t read_bin(const uint32_t *bin) {
  return __hip_atomic_load(global(bin), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void clear_bin(uint32_t *bin) {
  __hip_atomic_store(global(bin), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void put_candidate(unsigned long long *c, unsigned long long v) {
  __hip_atomic_store(global(c), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long get_candidate(const unsigned long long *c) {
  return __hip_atomic_load(global(c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// Run by the whole last workgroup of a pass: move the merged histogram into
// LDS (leaving the state's zero for the next pass), then the workgroup scans it
// from the largest digit down (keys) or the smallest up (indices) and fixes
// the digit that holds the need-th element.  `first`: the first pass of its kind
// (its prefix starts empty; the first key pass needs kk elements); `decide`:
// the second key pass, which chooses between gathering and the remaining
// radix passes; `last`: the final key pass, which also sets up the tie passes
// and the compaction.
template <bool KEYS>
__device__ void select_digit(const TopkJob &job, uint32_t *lh, int shift, int width, bool first, bool decide,
                             bool last) {
  TopkState *st = job.st;
  const int nb = 1 << width;
  // The whole table, without branches, so that the loads are in flight
  // together: bins at and above nb are zero (no pass leaves a bin set).
  constexpr int PER = TOPK_HIST / HIST_THREADS;
  uint32_t h[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) h[m] = read_bin(&st->hist[threadIdx.x + m * HIST_THREADS]);
#pragma unroll
  for (int m = 0; m < PER; ++m) lh[threadIdx.x + m * HIST_THREADS] = h[m];
#pragma unroll
  for (int m = 0; m < PER; ++m) clear_bin(&st->hist[threadIdx.x + m * HIST_THREADS]);
  if (threadIdx.x == 0) clear_bin(&st->done);
  __syncthreads();
  // every thread takes `per` consecutive ordinals; a block-wide scan of their
  // counts finds the thread whose ordinals hold the need-th element
  __shared__ uint32_t wave_total[HIST_THREADS / 64];
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int per = (nb + HIST_THREADS - 1) / HIST_THREADS;
  // ordinal o = threadIdx.x*per + i  <->  digit (KEYS ? nb-1-o : o)
  uint32_t mine = 0;
  for (int i = 0; i < per; ++i) {
    const int o = (int)threadIdx.x * per + i;
    if (o < nb) mine += lh[KEYS ? nb - 1 - o : o];
  }
  uint32_t incl = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wave_total[wave] = incl;
  __syncthreads();
  for (int w = 0; w < wave; ++w) incl += wave_total[w];
  const uint32_t excl = incl - mine;
  const uint32_t need = KEYS ? (first ? job.kk : st->need) : st->idx_need;
  if (!(excl < need && need <= incl)) return;
  uint32_t before = excl;
  for (int i = 0; i < per; ++i) {
    const int o = (int)threadIdx.x * per + i;
    const int d = KEYS ? nb - 1 - o : o;
    const uint32_t h = lh[d];
    if (before + h >= need) {
      const uint32_t left = need - before;
      if (KEYS) {
        st->key_prefix = (first ? 0u : st->key_prefix) | ((uint32_t)d << shift);
        st->need = left;
        if (decide) {
          // h keys share the new prefix: if they and the winners fit in LDS,
          // the next pass gathers them and orders the winners (no further
          // digit, index or compaction pass has work)
          const uint32_t gather = h + job.kk <= (uint32_t)TOPK_GATHER ? 1u : 0u;
          st->gathered = gather;
          if (gather) {
            st->tie_mode = 0u;
            st->count = 0u;
            st->bcount = 0u;
          }
        }
        if (last) {
          st->eq_count = h;
          st->tie_mode = h > left ? 1u : 0u;
          st->idx_need = left;
          st->count = 0u;
        }
      } else {
        st->idx_prefix = (first ? 0u : st->idx_prefix) | ((uint32_t)d << shift);
        st->idx_need = left;
      }
      return;
    }
    before += h;
  }
}

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

// A word's place among nc distinct words is the number of larger words; each
// thread ranks M of them against all.
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
    if (i < nc) {
      job.vals[rank[m]] = key_value((uint32_t)(w[m] >> 32));
      job.idx[rank[m]] = (int64_t)(0xffffffffu - (uint32_t)(w[m] & 0xffffffffull));
    }
  }
  for (int i = nc + threadIdx.x; i < job.top_k; i += blockDim.x) {
    job.vals[i] = -__builtin_inff();
    job.idx[i] = -1;
  }
}

// Orders the nc distinct (key, index) words in s[0..nc) (LDS, room for cap
// words) in decreasing order and writes the outputs; the whole workgroup
// calls it.  Up to RANK_SORT_MAX words by rank counting, above by a bitonic
// network over the next power of two.
__device__ void order_and_write(const TopkJob &job, unsigned long long *s, int nc, int cap) {
  if (nc <= HIST_THREADS) return rank_and_write<1>(job, s, nc, cap);
  if (nc <= 2 * HIST_THREADS) return rank_and_write<2>(job, s, nc, cap);
  if (nc <= RANK_SORT_MAX) return rank_and_write<RANK_SORT_MAX / HIST_THREADS>(job, s, nc, cap);
  int p2 = 1;
  while (p2 < nc) p2 <<= 1;
  for (int i = nc + threadIdx.x; i < p2; i += blockDim.x) s[i] = 0ull;
  __syncthreads();
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
  if (!finish_pass(st, 0, js.lb, js.nblk)) return;
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
  if (job.kk == 0) return;
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
  if (finish_pass(job.st, nb, js.lb, js.nblk))
    select_digit<true>(job, lh, shift, width, pass == 0, pass == 1, pass == 2);
}

// Index pass: among keys equal to the threshold, histogram of index digit
// [shift, shift+width) of the indices that match the index prefix so far.
__global__ __launch_bounds__(HIST_THREADS) void topk_index_pass_kernel(TopkJobs J, int shift, int width, int first) {
  const JobShare js = job_of(J);
  const TopkJob &job = js.job;
  if (job.kk == 0 || job.st->tie_mode == 0u) return;
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
  if (finish_pass(job.st, nb, js.lb, js.nblk)) select_digit<false>(job, lh, shift, width, first != 0, false, false);
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
  if (!finish_pass(st, 0, js.lb, js.nblk)) return;
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
  return job;
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
  const int64_t target = (int64_t)cu_count * 8;
  const int64_t chunk = std::max<int64_t>(kMinShare, (total_n + target - 1) / target);
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

hipError_t launch_topk_jobs(const TopkJobs &J, int64_t total_blocks, int64_t max_n, hipStream_t stream) {
  if (total_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_blocks), block(HIST_THREADS);
  static const int key_shift[3] = {20, 10, 0}, key_width[3] = {12, 10, 10};
  for (int pass = 0; pass < 3; ++pass)
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
                       hipStream_t stream) {
  if (top_k <= 0) return hipSuccess;
  TopkJobs J;
  J.jobs = nullptr;
  J.block_job = nullptr;
  J.single = make_topk_job(stat, n, top_k, vals, idx, ws);
  const int64_t blocks = topk_assign_blocks(&J.single, 1, cu_count);
  return launch_topk_jobs(J, blocks, n, stream);
}

}  // namespace emri
