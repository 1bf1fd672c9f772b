// Exact, deterministic top-k of the statistic vector (Sec. II D keeps the
// best-scoring candidates of a batch).  Order: decreasing S, then increasing
// template index; NaN ranks below every number and -0 equals +0.
//
// Radix select on an order-preserving 32-bit key of S: three histogram passes
// (11, 11 and 10 bits) find the key T of the k-th element and how many of the
// elements equal to T belong to the top-k.  If T is shared by more elements
// than are needed, three more passes select the needed count of smallest
// template indices among them.  One compaction pass then gathers exactly k
// (key, index) pairs, and one workgroup sorts them with a bitonic network in
// LDS.  All passes stream the statistic with 16-byte loads; histograms are
// built in LDS and merged with one atomic per non-empty bin per workgroup.
#include <hip/hip_runtime.h>

#include "common.h"
#include "score_internal.h"

namespace emri {
namespace {

constexpr int HIST_THREADS = 256;

__device__ __forceinline__ uint32_t order_key(float v) {
  uint32_t u = __float_as_uint(v);
  if (v != v) return 0u;                       // NaN: lowest
  if (u == 0x80000000u) u = 0u;                // -0 -> +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Digit layout: keys use (shift, width) = (21,11), (10,11), (0,10);
// indices (31-bit) use (20,11), (10,10), (0,10).
__device__ __forceinline__ void key_digit(int pass, int *shift, int *width) {
  *shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
  *width = pass == 2 ? 10 : 11;
}
__device__ __forceinline__ void idx_digit(int pass, int *shift, int *width) {
  *shift = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
  *width = pass == 0 ? 11 : 10;
}

template <typename F>
__device__ __forceinline__ void for_each_stat(const float *__restrict__ stat, int64_t n, F &&f) {
  const int64_t n4 = n >> 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
    const float4 v = reinterpret_cast<const float4 *>(stat)[q];
    f(4 * q + 0, v.x);
    f(4 * q + 1, v.y);
    f(4 * q + 2, v.z);
    f(4 * q + 3, v.w);
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) f(i, stat[i]);
}

__device__ __forceinline__ void flush_hist(uint32_t *lh, uint32_t *gh) {
  __syncthreads();
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x)
    if (lh[b]) atomicAdd(&gh[b], lh[b]);
}

__global__ __launch_bounds__(256) void topk_init_kernel(TopkState *st, uint32_t kk) {
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x) st->hist[b] = 0u;
  if (threadIdx.x == 0) {
    st->key_prefix = 0u;
    st->need = kk;
    st->idx_prefix = 0u;
    st->idx_need = 0u;
    st->tie_mode = 0u;
    st->count = 0u;
    st->eq_count = 0u;
  }
}

__global__ __launch_bounds__(HIST_THREADS) void topk_hist_key_kernel(const float *__restrict__ stat, int64_t n,
                                                                     TopkState *st, int pass) {
  __shared__ uint32_t lh[TOPK_HIST];
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x) lh[b] = 0u;
  __syncthreads();
  int shift, width;
  key_digit(pass, &shift, &width);
  const int hi = shift + width;
  const uint32_t prefix = st->key_prefix;
  const uint32_t mask = (1u << width) - 1u;
  for_each_stat(stat, n, [&](int64_t, float v) {
    const uint32_t k = order_key(v);
    if (hi >= 32 || (k >> hi) == (prefix >> hi)) atomicAdd(&lh[(k >> shift) & mask], 1u);
  });
  flush_hist(lh, st->hist);
}

// One wave scans the histogram from the largest digit down (keys) or from the
// smallest up (indices) and fixes the digit holding the need-th element.
template <bool KEYS>
__global__ __launch_bounds__(64) void topk_select_kernel(TopkState *st, int pass) {
  if (!KEYS && st->tie_mode == 0u) return;
  int shift, width;
  if (KEYS) key_digit(pass, &shift, &width); else idx_digit(pass, &shift, &width);
  const int nb = 1 << width;
  const int per = nb / 64;
  const int lane = threadIdx.x;
  // ordinal o = lane*per + i  <->  digit (KEYS ? nb-1-o : o)
  uint32_t mine = 0;
  for (int i = 0; i < per; ++i) {
    const int o = lane * per + i;
    mine += st->hist[KEYS ? nb - 1 - o : o];
  }
  uint32_t incl = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  const uint32_t excl = incl - mine;
  const uint32_t need = KEYS ? st->need : st->idx_need;
  const bool owner = excl < need && need <= incl;
  if (owner) {
    uint32_t before = excl;
    for (int i = 0; i < per; ++i) {
      const int o = lane * per + i;
      const int d = KEYS ? nb - 1 - o : o;
      const uint32_t h = st->hist[d];
      if (before + h >= need) {
        const uint32_t left = need - before;
        if (KEYS) {
          st->key_prefix |= (uint32_t)d << shift;
          st->need = left;
          if (pass == 2) {
            st->eq_count = h;
            st->tie_mode = h > left ? 1u : 0u;
            st->idx_need = left;
          }
        } else {
          st->idx_prefix |= (uint32_t)d << shift;
          st->idx_need = left;
        }
        break;
      }
      before += h;
    }
  }
  __syncthreads();
  for (int b = lane; b < nb; b += 64) st->hist[b] = 0u;
}

__global__ __launch_bounds__(HIST_THREADS) void topk_hist_idx_kernel(const float *__restrict__ stat, int64_t n,
                                                                     TopkState *st, int pass) {
  if (st->tie_mode == 0u) return;
  __shared__ uint32_t lh[TOPK_HIST];
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x) lh[b] = 0u;
  __syncthreads();
  int shift, width;
  idx_digit(pass, &shift, &width);
  const int hi = shift + width;
  const uint32_t key = st->key_prefix;
  const uint32_t prefix = st->idx_prefix;
  const uint32_t mask = (1u << width) - 1u;
  for_each_stat(stat, n, [&](int64_t i, float v) {
    const uint32_t u = (uint32_t)i;
    if (order_key(v) == key && (hi >= 31 || (u >> hi) == (prefix >> hi))) atomicAdd(&lh[(u >> shift) & mask], 1u);
  });
  flush_hist(lh, st->hist);
}

__global__ __launch_bounds__(HIST_THREADS) void topk_compact_kernel(const float *__restrict__ stat, int64_t n,
                                                                    TopkState *st, unsigned long long *cand,
                                                                    uint32_t kk) {
  const uint32_t key = st->key_prefix;
  const bool tie = st->tie_mode != 0u;
  const uint32_t thr = st->idx_prefix;
  for_each_stat(stat, n, [&](int64_t i, float v) {
    const uint32_t k = order_key(v);
    const bool sel = k > key || (k == key && (!tie || (uint32_t)i <= thr));
    if (sel) {
      const uint32_t pos = atomicAdd(&st->count, 1u);
      if (pos < kk) cand[pos] = ((unsigned long long)k << 32) | (unsigned long long)(0xffffffffu - (uint32_t)i);
    }
  });
}

__global__ __launch_bounds__(1024) void topk_final_kernel(const unsigned long long *cand, uint32_t kk, int top_k,
                                                          float *vals, int64_t *idx) {
  __shared__ unsigned long long s[EMRI_MAX_TOPK];
  int p2 = 1;
  while (p2 < (int)kk) p2 <<= 1;
  for (int i = threadIdx.x; i < p2; i += blockDim.x) s[i] = i < (int)kk ? cand[i] : 0ull;
  __syncthreads();
  // bitonic sort, descending
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
  for (int i = threadIdx.x; i < top_k; i += blockDim.x) {
    if (i < (int)kk) {
      const unsigned long long c = s[i];
      vals[i] = key_value((uint32_t)(c >> 32));
      idx[i] = (int64_t)(0xffffffffu - (uint32_t)(c & 0xffffffffull));
    } else {
      vals[i] = -__builtin_inff();
      idx[i] = -1;
    }
  }
}

}  // namespace

size_t topk_workspace_bytes(int top_k) {
  return round_up(sizeof(TopkState), 256) + round_up((size_t)(top_k > 0 ? top_k : 1) * 8, 256);
}

hipError_t launch_topk(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws, int cu_count,
                       hipStream_t stream) {
  if (top_k <= 0) return hipSuccess;
  TopkState *st = reinterpret_cast<TopkState *>(ws);
  unsigned long long *cand =
      reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) + round_up(sizeof(TopkState), 256));
  const uint32_t kk = (uint32_t)(n < (int64_t)top_k ? n : (int64_t)top_k);
  if (kk > 0) {
    const int64_t work = (n + 4 * HIST_THREADS - 1) / (4 * HIST_THREADS);
    const int grid = (int)(work < (int64_t)cu_count * 4 ? (work > 0 ? work : 1) : (int64_t)cu_count * 4);
    hipLaunchKernelGGL(topk_init_kernel, dim3(1), dim3(256), 0, stream, st, kk);
    for (int pass = 0; pass < 3; ++pass) {
      hipLaunchKernelGGL(topk_hist_key_kernel, dim3(grid), dim3(HIST_THREADS), 0, stream, stat, n, st, pass);
      hipLaunchKernelGGL(topk_select_kernel<true>, dim3(1), dim3(64), 0, stream, st, pass);
    }
    for (int pass = 0; pass < 3; ++pass) {
      hipLaunchKernelGGL(topk_hist_idx_kernel, dim3(grid), dim3(HIST_THREADS), 0, stream, stat, n, st, pass);
      hipLaunchKernelGGL(topk_select_kernel<false>, dim3(1), dim3(64), 0, stream, st, pass);
    }
    hipLaunchKernelGGL(topk_compact_kernel, dim3(grid), dim3(HIST_THREADS), 0, stream, stat, n, st, cand, kk);
  }
  hipLaunchKernelGGL(topk_final_kernel, dim3(1), dim3(1024), 0, stream, cand, kk, top_k, vals, idx);
  return hipGetLastError();
}

}  // namespace emri
