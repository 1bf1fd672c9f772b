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

// The job of this workgroup: blockIdx.y indexes the job table, or the single
// job passed by value when there is no table.
__device__ __forceinline__ TopkJob job_of(const TopkJobs &J) {
  if (J.jobs == nullptr) return J.single;
  return load_uniform(J.jobs + blockIdx.y);
}

__global__ __launch_bounds__(256) void topk_init_kernel(TopkJobs J) {
  const TopkJob job = job_of(J);
  TopkState *st = job.st;
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x) st->hist[b] = 0u;
  if (threadIdx.x == 0) {
    st->key_prefix = 0u;
    st->need = job.kk;
    st->idx_prefix = 0u;
    st->idx_need = 0u;
    st->tie_mode = 0u;
    st->count = 0u;
    st->eq_count = 0u;
  }
}

__global__ __launch_bounds__(HIST_THREADS) void topk_hist_key_kernel(TopkJobs J, int pass) {
  const TopkJob job = job_of(J);
  if (job.kk == 0) return;
  __shared__ uint32_t lh[TOPK_HIST];
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x) lh[b] = 0u;
  __syncthreads();
  int shift, width;
  key_digit(pass, &shift, &width);
  const int hi = shift + width;
  const uint32_t prefix = job.st->key_prefix;
  const uint32_t mask = (1u << width) - 1u;
  for_each_stat(job.stat, job.n, [&](int64_t, float v) {
    const uint32_t k = order_key(v);
    if (hi >= 32 || (k >> hi) == (prefix >> hi)) atomicAdd(&lh[(k >> shift) & mask], 1u);
  });
  flush_hist(lh, job.st->hist);
}

// One wave scans the histogram from the largest digit down (keys) or from the
// smallest up (indices) and fixes the digit holding the need-th element.
template <bool KEYS>
__global__ __launch_bounds__(64) void topk_select_kernel(TopkJobs J, int pass) {
  const TopkJob job = job_of(J);
  TopkState *st = job.st;
  if (job.kk == 0) return;
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

__global__ __launch_bounds__(HIST_THREADS) void topk_hist_idx_kernel(TopkJobs J, int pass) {
  const TopkJob job = job_of(J);
  if (job.kk == 0 || job.st->tie_mode == 0u) return;
  __shared__ uint32_t lh[TOPK_HIST];
  for (int b = threadIdx.x; b < TOPK_HIST; b += blockDim.x) lh[b] = 0u;
  __syncthreads();
  int shift, width;
  idx_digit(pass, &shift, &width);
  const int hi = shift + width;
  const uint32_t key = job.st->key_prefix;
  const uint32_t prefix = job.st->idx_prefix;
  const uint32_t mask = (1u << width) - 1u;
  for_each_stat(job.stat, job.n, [&](int64_t i, float v) {
    const uint32_t u = (uint32_t)i;
    if (order_key(v) == key && (hi >= 31 || (u >> hi) == (prefix >> hi))) atomicAdd(&lh[(u >> shift) & mask], 1u);
  });
  flush_hist(lh, job.st->hist);
}

__global__ __launch_bounds__(HIST_THREADS) void topk_compact_kernel(TopkJobs J) {
  const TopkJob job = job_of(J);
  if (job.kk == 0) return;
  TopkState *st = job.st;
  const uint32_t key = st->key_prefix;
  const bool tie = st->tie_mode != 0u;
  const uint32_t thr = st->idx_prefix;
  const uint32_t kk = job.kk;
  unsigned long long *cand = job.cand;
  for_each_stat(job.stat, job.n, [&](int64_t i, float v) {
    const uint32_t k = order_key(v);
    const bool sel = k > key || (k == key && (!tie || (uint32_t)i <= thr));
    if (sel) {
      const uint32_t pos = atomicAdd(&st->count, 1u);
      if (pos < kk) cand[pos] = ((unsigned long long)k << 32) | (unsigned long long)(0xffffffffu - (uint32_t)i);
    }
  });
}

__global__ __launch_bounds__(1024) void topk_final_kernel(TopkJobs J) {
  const TopkJob job = job_of(J);
  __shared__ unsigned long long s[EMRI_MAX_TOPK];
  const int kk = (int)job.kk;
  int p2 = 1;
  while (p2 < kk) p2 <<= 1;
  for (int i = threadIdx.x; i < p2; i += blockDim.x) s[i] = i < kk ? job.cand[i] : 0ull;
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

}  // namespace

size_t topk_workspace_bytes(int top_k) {
  return round_up(sizeof(TopkState), 256) + round_up((size_t)(top_k > 0 ? top_k : 1) * 8, 256);
}

TopkJob make_topk_job(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws) {
  TopkJob job;
  job.stat = stat;
  job.n = n;
  job.top_k = top_k;
  job.kk = (uint32_t)(n < (int64_t)top_k ? n : (int64_t)top_k);
  job.st = reinterpret_cast<TopkState *>(ws);
  job.cand = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) + round_up(sizeof(TopkState), 256));
  job.vals = vals;
  job.idx = idx;
  return job;
}

hipError_t launch_topk_jobs(const TopkJobs &J, int n_jobs, int64_t max_n, int cu_count, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  const int64_t work = (max_n + 4 * HIST_THREADS - 1) / (4 * HIST_THREADS);
  const int gx = (int)(work < (int64_t)cu_count * 4 ? (work > 0 ? work : 1) : (int64_t)cu_count * 4);
  const dim3 one(1, n_jobs), hist(gx, n_jobs);
  hipLaunchKernelGGL(topk_init_kernel, one, dim3(256), 0, stream, J);
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(topk_hist_key_kernel, hist, dim3(HIST_THREADS), 0, stream, J, pass);
    hipLaunchKernelGGL(topk_select_kernel<true>, one, dim3(64), 0, stream, J, pass);
  }
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(topk_hist_idx_kernel, hist, dim3(HIST_THREADS), 0, stream, J, pass);
    hipLaunchKernelGGL(topk_select_kernel<false>, one, dim3(64), 0, stream, J, pass);
  }
  hipLaunchKernelGGL(topk_compact_kernel, hist, dim3(HIST_THREADS), 0, stream, J);
  hipLaunchKernelGGL(topk_final_kernel, one, dim3(1024), 0, stream, J);
  return hipGetLastError();
}

hipError_t launch_topk(const float *stat, int64_t n, int top_k, float *vals, int64_t *idx, void *ws, int cu_count,
                       hipStream_t stream) {
  if (top_k <= 0) return hipSuccess;
  TopkJobs J;
  J.jobs = nullptr;
  J.single = make_topk_job(stat, n, top_k, vals, idx, ws);
  return launch_topk_jobs(J, 1, n, cu_count, stream);
}

}  // namespace emri
