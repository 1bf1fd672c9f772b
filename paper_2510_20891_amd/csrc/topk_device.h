// Device building blocks of the top-k passes (radix digits of an
// order-preserving key, LDS histograms, the two-level merge and the digit
// selection), shared by the top-k kernels and the scoring kernel, which can
// run the first key pass over its own statistics.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

template <int THREADS>
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
    constexpr int PER = TOPK_HIST / THREADS;
    uint32_t h[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) h[m] = read_bin(&st->ghist[g][threadIdx.x + m * THREADS]);
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int w = threadIdx.x + m * THREADS;
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

// Run by the whole last workgroup of a pass: move the merged histogram into
// LDS (leaving the state's zero for the next pass), then the workgroup scans it
// from the largest digit down (keys) or the smallest up (indices) and fixes
// the digit that holds the need-th element.  `first`: the first pass of its kind
// (its prefix starts empty; the first key pass needs kk elements, or
// first_need if that is not zero); `decide`:
// the second key pass, which chooses between gathering and the remaining
// radix passes; `last`: the final key pass, which also sets up the tie passes
// and the compaction.
template <bool KEYS, int THREADS>
__device__ void select_digit(const TopkJob &job, uint32_t *lh, int shift, int width, bool first, bool decide,
                             bool last, uint32_t first_need = 0u) {
  TopkState *st = job.st;
  const int nb = 1 << width;
  // The whole table, without branches, so that the loads are in flight
  // together: bins at and above nb are zero (no pass leaves a bin set).
  constexpr int PER = TOPK_HIST / THREADS;
  uint32_t h[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) h[m] = read_bin(&st->hist[threadIdx.x + m * THREADS]);
#pragma unroll
  for (int m = 0; m < PER; ++m) lh[threadIdx.x + m * THREADS] = h[m];
#pragma unroll
  for (int m = 0; m < PER; ++m) clear_bin(&st->hist[threadIdx.x + m * THREADS]);
  if (threadIdx.x == 0) clear_bin(&st->done);
  __syncthreads();
  // every thread takes `per` consecutive ordinals; a block-wide scan of their
  // counts finds the thread whose ordinals hold the need-th element
  __shared__ uint32_t wave_total[THREADS / 64];
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int per = (nb + THREADS - 1) / THREADS;
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
  const uint32_t need = KEYS ? (first ? (first_need ? first_need : job.kk) : st->need) : st->idx_need;
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

}  // namespace
}  // namespace emri
