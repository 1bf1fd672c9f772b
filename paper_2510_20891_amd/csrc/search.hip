// Population search over basis coefficients (Sec. II D): seeding and the
// track-space differential-evolution generation of Eq. (11), for many chains
// at once (a chain is one population against one spectrogram and basis; the
// progressive-duration search runs one chain per observed duration).
//
// One generation is two launches (search_generation), or, for a pair of
// generations, one launch each (search_generations, with a second copy of
// the population in the workspace), all reading device tables written by
// search_plan, so generations can be captured into a HIP graph:
//   1. de_trial_score_kernel: per walker (eight lanes each), the trial track
//      f_trial = f + F (f_r1 - f_r2) is formed segment by segment in FP64
//      (f = f0 + U c), projected back onto the basis with its pseudo-inverse,
//      c_trial = pinv(U) (f_trial - f0), rounded to FP32 (a chain's basis
//      rows are a time-shifted part of the one-year basis, no longer
//      orthonormal; the plan computes each chain's pseudo-inverse on the
//      host, FP64 one-sided Jacobi, and keeps it in the workspace), and
//      scored with power gathered from the spectrogram in place;
//   2. de_select_kernel: a trial inside the prior box (bounds included) whose
//      statistic is strictly higher replaces the walker.
// Walkers whose partner indices are out of range or not distinct keep their
// current vector (their trial is never accepted).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <utility>
#include <vector>

#include "common.h"
#include "score_internal.h"

using namespace emri;

namespace {

constexpr uint32_t kSearchMagic = 0x45534348u;   // "ESCH"

template <typename T>
struct type_tag {
  using type = T;
};
constexpr int kSearchThreads = 256;

// One chain as the kernels see it (device table).
struct ChainDesc {
  const double *f0, *U, *box_lo, *box_hi;
  const double *pinvt;             // pinv(U) transposed: n_seg x K (workspace)
  float *coeffs, *stat;            // the walkers (updated in place)
  float *coeffs_b, *stat_b;        // second copy of the population (workspace), for fused generations
  float *trial, *trial_stat;       // this generation's trials (workspace)
  const void *power;               // spectrogram rows (FP32 or FP16)
  double t_sft;
  int64_t offset;                  // first walker of the chain in the concatenated draws
  int32_t n_seg, n_walkers;
  int32_t pitch;                   // elements between spectrogram rows
  int32_t k_min, k_max;
  int32_t pad;
};

// What search_generation needs, kept in the caller's emri_search_plan.
struct SearchPlanData {
  uint32_t magic;
  int32_t n_chains;
  int32_t K;
  int32_t max_walkers;
  int32_t max_seg;
  int32_t dtype;
  const ChainDesc *chains;
  int64_t total_walkers;
};
static_assert(sizeof(SearchPlanData) <= sizeof(emri_search_plan), "search plan does not fit");

// f[alpha] of a walker (FP64): f0[alpha] + sum_k U[alpha, k] c_k
template <int K>
__device__ __forceinline__ double track_at(const double *f0, const double *Ua, const double (&c)[K], int alpha) {
  double f = f0[alpha];
#pragma unroll
  for (int k = 0; k < K; ++k) f = __builtin_fma(Ua[k], c[k], f);
  return f;
}

// The chain's basis rows (f0, U and the transposed pseudo-inverse), staged
// in LDS when they fit (every lane reads every row), else read in place.  In
// LDS a row of K doubles is padded to an odd number of doubles, so that the
// eight different rows the eight lanes of a walker read at once fall in
// different banks.
struct BasisRows {
  const double *f0, *U, *P;
  int stride;                      // doubles between consecutive rows of U and P
};

__host__ __device__ constexpr int padded_stride(int K) { return (K % 2 == 0) ? K + 1 : K; }

template <bool STAGE, int NT = kSearchThreads>
__device__ __forceinline__ BasisRows basis_rows(const ChainDesc &ch, int K, double *lds) {
  if constexpr (!STAGE) {
    return BasisRows{ch.f0, ch.U, ch.pinvt, K};
  } else {
    // f0 | U rows | pinv^T rows, eight loads in flight per lane before their stores
    const int n = ch.n_seg, nk = n * K, total = n + 2 * nk, ps = padded_stride(K);
    double *f0s = lds, *Us = lds + n, *Ps = lds + n + (size_t)n * ps;
    constexpr int D = 8;
    for (int e0 = threadIdx.x; e0 < total; e0 += D * NT) {
      double v[D];
#pragma unroll
      for (int u = 0; u < D; ++u) {
        const int e = e0 + u * NT;
        v[u] = e < n ? ch.f0[e] : (e < n + nk ? ch.U[e - n] : (e < total ? ch.pinvt[e - n - nk] : 0.0));
      }
#pragma unroll
      for (int u = 0; u < D; ++u) {
        const int e = e0 + u * NT;
        if (e < n) {
          f0s[e] = v[u];
        } else if (e < n + nk) {
          const int q = e - n;
          Us[(q / K) * ps + q % K] = v[u];
        } else if (e < total) {
          const int q = e - n - nk;
          Ps[(q / K) * ps + q % K] = v[u];
        }
      }
    }
    __syncthreads();
    return BasisRows{f0s, Us, Ps, ps};
  }
}

__global__ __launch_bounds__(kSearchThreads) void de_select_kernel(const ChainDesc *__restrict__ chains, int K,
                                                                   int32_t *__restrict__ accepted) {
  const ChainDesc ch = load_uniform(chains + blockIdx.y);
  const int i = blockIdx.x * kSearchThreads + threadIdx.x;
  if (i >= ch.n_walkers) return;
  bool inside = true;
  for (int k = 0; k < K; ++k) {
    const double v = (double)ch.trial[(size_t)i * K + k];
    inside &= v >= ch.box_lo[k] && v <= ch.box_hi[k];            // NaN: outside
  }
  const float s = ch.trial_stat[i];
  const bool take = inside && s > ch.stat[i];
  if (take) {
    for (int k = 0; k < K; ++k) ch.coeffs[(size_t)i * K + k] = ch.trial[(size_t)i * K + k];
    ch.stat[i] = s;
  }
  if (accepted) accepted[ch.offset + i] = take ? 1 : 0;
}

// One generation's trials.  Eight lanes work on one walker: lane s takes
// segments s, s + 8, s + 16, ...; the projection's partial sums and the
// statistic's partial sums are combined across the lanes with shuffles in a
// fixed order.  The trial's coefficients are rounded to FP32 (the walkers'
// representation) before its positions are evaluated in FP64 as in
// score_tracks, x = f0 T + sum_k c_k (U T)[alpha, k], rounded to the nearest
// bin (half to even); the power is gathered from the spectrogram in place (a
// population of a few hundred walkers reads too few elements of a row to pay
// for staging rows in LDS), up to 32 gathers per lane in flight at once.
// Each lane sums its segments in FP32 runs of 8 and in FP64 across runs and
// lanes.
//
// de_trial_score_kernel writes the trials and de_select_kernel selects
// afterwards (the population is only read meanwhile); de_generation_kernel
// does both in one launch, reading one copy of the population and writing
// the other (DIR 0: the chain's arrays to the workspace copy, DIR 1 back),
// so that every trial still sees the population of the previous generation.
constexpr int kLanesPerWalker = 8;      // measured: 16 lanes and 512 threads 33 us, 8 and 256 27 us
constexpr int kTrialThreads = 256;
constexpr int kWalkersPerBlock = kTrialThreads / kLanesPerWalker;
constexpr int kGatherRun = 32;          // gathers per lane in flight (one run covers 256 segments)

template <typename PT>
__device__ __forceinline__ float power_at(const void *p, size_t at);
template <>
__device__ __forceinline__ float power_at<float>(const void *p, size_t at) {
  return reinterpret_cast<const float *>(p)[at];
}
template <>
__device__ __forceinline__ float power_at<__half>(const void *p, size_t at) {
  return (float)__builtin_bit_cast(_Float16, reinterpret_cast<const unsigned short *>(p)[at]);
}

// Trial of walker i of a chain whose population is pop (FP32, n_walkers x K):
// its FP32 coefficients ct (NaN when the partners are invalid) and its
// statistic (identical in every lane of the walker; -inf when invalid).
template <int K, typename PT>
__device__ __forceinline__ float trial_of(const ChainDesc &ch, const BasisRows &B, const float *__restrict__ pop,
                                          int i, int sub, int a, int b, bool valid, double w, float (&ct)[K]) {
  double ci[K], ca[K], cb[K], out[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ci[k] = (double)pop[(size_t)i * K + k];
    ca[k] = valid ? (double)pop[(size_t)a * K + k] : ci[k];
    cb[k] = valid ? (double)pop[(size_t)b * K + k] : ci[k];
    out[k] = 0.0;
  }
  for (int alpha = sub; alpha < ch.n_seg; alpha += kLanesPerWalker) {
    const double *Ua = B.U + (size_t)alpha * B.stride;
    const double fi = track_at<K>(B.f0, Ua, ci, alpha);
    const double fa = track_at<K>(B.f0, Ua, ca, alpha);
    const double fb = track_at<K>(B.f0, Ua, cb, alpha);
    const double d = __builtin_fma(w, fa - fb, fi) - B.f0[alpha];     // f_trial - f0
    const double *Pa = B.P + (size_t)alpha * B.stride;
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = __builtin_fma(Pa[k], d, out[k]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = out[k];
#pragma unroll
    for (int off = kLanesPerWalker / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanesPerWalker);
    ct[k] = valid ? (float)v : __builtin_nanf("");
  }
  // the trial's statistic: a run's bins first, then its gathers in flight
  // together, then FP32 runs of 8 segments summed into FP64
  const double T = ch.t_sft;
  double sum = 0.0;
  for (int base = 0; base < ch.n_seg; base += kGatherRun * kLanesPerWalker) {
    // slots u < n_run hold a segment for some lane of the walker (wave-uniform)
    const int left = (ch.n_seg - base + kLanesPerWalker - 1) / kLanesPerWalker;
    const int n_run = left < kGatherRun ? left : kGatherRun;
    unsigned at[kGatherRun];
    bool in[kGatherRun];
    float v[kGatherRun];
#pragma unroll
    for (int u = 0; u < kGatherRun; ++u) {
      in[u] = false;
      v[u] = 0.0f;
      if (u < n_run) {
        const int alpha = base + sub + u * kLanesPerWalker;
        const int ar = alpha < ch.n_seg ? alpha : sub;
        const double *Ua = B.U + (size_t)ar * B.stride;
        double x = B.f0[ar] * T;
#pragma unroll
        for (int k = 0; k < K; ++k) x = __builtin_fma((double)ct[k], Ua[k] * T, x);
        const bool finite = __builtin_fabs(x) < 67108864.0;              // 2^26 bins; NaN fails
        const int bin = finite ? (int)__builtin_rint(x) : -1;
        in[u] = alpha < ch.n_seg && finite && bin >= ch.k_min && bin <= ch.k_max;
        at[u] = (unsigned)ar * (unsigned)ch.pitch + (unsigned)(in[u] ? bin : ch.k_min);
      }
    }
#pragma unroll
    for (int u = 0; u < kGatherRun; ++u)
      if (u < n_run) v[u] = power_at<PT>(ch.power, at[u]);
#pragma unroll
    for (int r = 0; r < kGatherRun; r += 8) {
      if (r < n_run) {
        float acc = 0.0f;
#pragma unroll
        for (int u = r; u < r + 8; ++u) acc += in[u] ? v[u] : 0.0f;
        sum += (double)acc;
      }
    }
  }
#pragma unroll
  for (int off = kLanesPerWalker / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kLanesPerWalker);
  return valid ? (float)sum : -__builtin_inff();
}

struct WalkerSlot {
  int i, sub, a, b;
  bool live, valid;
  double w;
};

__device__ __forceinline__ WalkerSlot walker_slot(const ChainDesc &ch, const int32_t *r1, const int32_t *r2,
                                                  const double *F) {
  WalkerSlot ws;
  ws.sub = (int)(threadIdx.x & (kLanesPerWalker - 1));
  const int i_raw = blockIdx.x * kWalkersPerBlock + (int)(threadIdx.x / kLanesPerWalker);
  ws.live = i_raw < ch.n_walkers;
  ws.i = ws.live ? i_raw : 0;                      // idle lanes compute walker 0 and store nothing
  const int64_t gi = ch.offset + ws.i;
  ws.a = r1[gi];
  ws.b = r2[gi];
  ws.valid = ws.a >= 0 && ws.a < ch.n_walkers && ws.b >= 0 && ws.b < ch.n_walkers && ws.a != ws.i &&
             ws.b != ws.i && ws.a != ws.b;
  ws.w = ws.valid ? F[gi] : 0.0;
  return ws;
}

template <int K, bool STAGE, typename PT>
__global__ __launch_bounds__(kTrialThreads) void de_trial_score_kernel(const ChainDesc *__restrict__ chains,
                                                                        const int32_t *__restrict__ r1,
                                                                        const int32_t *__restrict__ r2,
                                                                        const double *__restrict__ F) {
  extern __shared__ double stage_rows[];
  const ChainDesc ch = load_uniform(chains + blockIdx.y);
  if ((int)(blockIdx.x * kWalkersPerBlock) >= ch.n_walkers) return;    // whole workgroup idle
  const BasisRows B = basis_rows<STAGE, kTrialThreads>(ch, K, stage_rows);
  const WalkerSlot ws = walker_slot(ch, r1, r2, F);
  float ct[K];
  const float ts = trial_of<K, PT>(ch, B, ch.coeffs, ws.i, ws.sub, ws.a, ws.b, ws.valid, ws.w, ct);
  if (ws.live) {
    for (int k = ws.sub; k < K; k += kLanesPerWalker) {
#pragma unroll
      for (int q = 0; q < K; ++q)
        if (q == k) ch.trial[(size_t)ws.i * K + k] = ct[q];
    }
    if (ws.sub == 0) ch.trial_stat[ws.i] = ts;
  }
}

template <int K, bool STAGE, typename PT>
__global__ __launch_bounds__(kTrialThreads) void de_generation_kernel(const ChainDesc *__restrict__ chains,
                                                                       const int32_t *__restrict__ r1,
                                                                       const int32_t *__restrict__ r2,
                                                                       const double *__restrict__ F, int dir) {
  extern __shared__ double stage_rows[];
  const ChainDesc ch = load_uniform(chains + blockIdx.y);
  if ((int)(blockIdx.x * kWalkersPerBlock) >= ch.n_walkers) return;    // whole workgroup idle
  const BasisRows B = basis_rows<STAGE, kTrialThreads>(ch, K, stage_rows);
  const float *pop = dir == 0 ? ch.coeffs : ch.coeffs_b;
  const float *pstat = dir == 0 ? ch.stat : ch.stat_b;
  float *dst = dir == 0 ? ch.coeffs_b : ch.coeffs;
  float *dstat = dir == 0 ? ch.stat_b : ch.stat;
  const WalkerSlot ws = walker_slot(ch, r1, r2, F);
  float ct[K];
  const float ts = trial_of<K, PT>(ch, B, pop, ws.i, ws.sub, ws.a, ws.b, ws.valid, ws.w, ct);
  bool inside = true;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double v = (double)ct[k];
    inside &= v >= ch.box_lo[k] && v <= ch.box_hi[k];                  // NaN: outside
  }
  const float old = pstat[ws.i];
  const bool take = inside && ts > old;
  if (ws.live) {
    for (int k = ws.sub; k < K; k += kLanesPerWalker) {
#pragma unroll
      for (int q = 0; q < K; ++q)
        if (q == k) dst[(size_t)ws.i * K + k] = take ? ct[q] : pop[(size_t)ws.i * K + k];
    }
    if (ws.sub == 0) dstat[ws.i] = take ? ts : old;
  }
}

// Seeding: every candidate's track is moved by one constant so that its first
// segment sits at f_init, then projected back (FP32 result).  Chain c's
// candidates are draws[c * n_draw + j] (K values each); cand holds them at a
// stride of cand_stride floats per chain.
template <int K, bool STAGE>
__global__ __launch_bounds__(kSearchThreads) void seed_move_kernel(const ChainDesc *__restrict__ chains,
                                                                   const float *__restrict__ draws,
                                                                   const double *__restrict__ f_init, int n_draw,
                                                                   float *__restrict__ cand, int64_t cand_stride) {
  extern __shared__ double stage_rows[];
  const ChainDesc ch = load_uniform(chains + blockIdx.y);
  const BasisRows B = basis_rows<STAGE>(ch, K, stage_rows);
  const int j = blockIdx.x * kSearchThreads + threadIdx.x;
  if (j >= n_draw) return;
  const int64_t gj = (int64_t)blockIdx.y * n_draw + j;
  double c[K], out[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    c[k] = (double)draws[(size_t)gj * K + k];
    out[k] = 0.0;
  }
  const double shift = f_init[gj] - track_at<K>(B.f0, B.U, c, 0);
  for (int alpha = 0; alpha < ch.n_seg; ++alpha) {
    const double *Ua = B.U + (size_t)alpha * B.stride;
    const double d = (track_at<K>(B.f0, Ua, c, alpha) + shift) - B.f0[alpha];
    const double *Pa = B.P + (size_t)alpha * B.stride;
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = __builtin_fma(Pa[k], d, out[k]);
  }
  float *dst = cand + (size_t)blockIdx.y * cand_stride + (size_t)j * K;
#pragma unroll
  for (int k = 0; k < K; ++k) dst[k] = (float)out[k];
}

// The n_walkers best candidates of each chain become its walkers.
__global__ __launch_bounds__(kSearchThreads) void seed_gather_kernel(const ChainDesc *__restrict__ chains, int K,
                                                                     const float *__restrict__ cand,
                                                                     int64_t cand_stride,
                                                                     const float *__restrict__ top_val,
                                                                     const int64_t *__restrict__ top_idx,
                                                                     int64_t top_stride) {
  const ChainDesc ch = load_uniform(chains + blockIdx.y);
  const int i = blockIdx.x * kSearchThreads + threadIdx.x;
  if (i >= ch.n_walkers) return;
  const int64_t slot = (int64_t)blockIdx.y * top_stride + i;
  const int64_t j = top_idx[slot];                 // always a candidate: n_walkers <= n_draw
  const float *src = cand + (size_t)blockIdx.y * cand_stride + (size_t)(j >= 0 ? j : 0) * K;
  for (int k = 0; k < K; ++k) ch.coeffs[(size_t)i * K + k] = src[k];
  ch.stat[i] = top_val[slot];
}

// a ranks above b in the order (-S, index) with NaN below every number
__device__ __forceinline__ bool ranks_above(float va, int ia, float vb, int ib) {
  if (ib < 0) return ia >= 0;
  if (ia < 0) return false;
  const bool na = va != va, nb = vb != vb;
  if (na != nb) return nb;
  if (!na && va != vb) return va > vb;
  return ia < ib;
}

// Per chain: the best walker by (-S, index), and its statistic normalised by
// the chain's noise-only mean and standard deviation.
__global__ __launch_bounds__(kSearchThreads) void search_best_kernel(const ChainDesc *__restrict__ chains,
                                                                     const double *__restrict__ noise_mean,
                                                                     const double *__restrict__ noise_std,
                                                                     float *__restrict__ best_stat,
                                                                     int32_t *__restrict__ best_idx,
                                                                     double *__restrict__ best_norm) {
  __shared__ float sv[kSearchThreads];
  __shared__ int si[kSearchThreads];
  const ChainDesc ch = load_uniform(chains + blockIdx.x);
  float v = 0.0f;
  int idx = -1;
  for (int i = threadIdx.x; i < ch.n_walkers; i += kSearchThreads) {
    const float s = ch.stat[i];
    if (ranks_above(s, i, v, idx)) {
      v = s;
      idx = i;
    }
  }
  sv[threadIdx.x] = v;
  si[threadIdx.x] = idx;
  __syncthreads();
  for (int off = kSearchThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off && ranks_above(sv[threadIdx.x + off], si[threadIdx.x + off], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + off];
      si[threadIdx.x] = si[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    best_stat[blockIdx.x] = sv[0];
    best_idx[blockIdx.x] = si[0];
    if (best_norm)
      best_norm[blockIdx.x] = ((double)sv[0] - noise_mean[blockIdx.x]) / noise_std[blockIdx.x];
  }
}

// Mean and sample standard deviation (n - 1 in the denominator) over n_real
// realisations of each chain's best statistic; best[r * n_chains + c].
__global__ __launch_bounds__(kSearchThreads) void noise_moments_kernel(const float *__restrict__ best, int n_real,
                                                                       int n_chains, double *__restrict__ mean,
                                                                       double *__restrict__ sd) {
  const int c = blockIdx.x * kSearchThreads + threadIdx.x;
  if (c >= n_chains) return;
  double m = 0.0;
  for (int r = 0; r < n_real; ++r) m += (double)best[(size_t)r * n_chains + c];
  m /= n_real;
  double q = 0.0;
  for (int r = 0; r < n_real; ++r) {
    const double d = (double)best[(size_t)r * n_chains + c] - m;
    q += d * d;
  }
  mean[c] = m;
  sd[c] = __builtin_sqrt(q / (n_real - 1));
}

// Bytes of LDS that stage a chain of n_seg rows, or 0 when they do not fit
// (the kernels then read the rows in place).
constexpr size_t kStageLimit = 160 * 1024;
size_t stage_bytes(int max_seg, int K) {
  const size_t b = sizeof(double) * (size_t)max_seg * (2 * (size_t)padded_stride(K) + 1);
  return b <= kStageLimit ? b : 0;
}

template <int... Ks>
hipError_t launch_trial_score(int K, int dtype, int max_seg, dim3 grid, hipStream_t stream, const ChainDesc *chains,
                              const int32_t *r1, const int32_t *r2, const double *F,
                              std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  const size_t lds = stage_bytes(max_seg, K);
  auto one = [&](auto kc, auto pt) {
    constexpr int KK = decltype(kc)::value;
    using PT = typename decltype(pt)::type;
    auto kern = lds ? de_trial_score_kernel<KK, true, PT> : de_trial_score_kernel<KK, false, PT>;
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return;
    hipLaunchKernelGGL(kern, grid, dim3(kTrialThreads), lds, stream, chains, r1, r2, F);
    err = hipGetLastError();
  };
  if (dtype == EMRI_F32)
    ((K == Ks + 1 ? (one(std::integral_constant<int, Ks + 1>{}, type_tag<float>{}), true) : false) || ...);
  else
    ((K == Ks + 1 ? (one(std::integral_constant<int, Ks + 1>{}, type_tag<__half>{}), true) : false) || ...);
  return err;
}

template <int... Ks>
hipError_t launch_generation(int K, int dtype, int max_seg, dim3 grid, hipStream_t stream, const ChainDesc *chains,
                             const int32_t *r1, const int32_t *r2, const double *F, int dir,
                             std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  const size_t lds = stage_bytes(max_seg, K);
  auto one = [&](auto kc, auto pt) {
    constexpr int KK = decltype(kc)::value;
    using PT = typename decltype(pt)::type;
    auto kern = lds ? de_generation_kernel<KK, true, PT> : de_generation_kernel<KK, false, PT>;
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return;
    hipLaunchKernelGGL(kern, grid, dim3(kTrialThreads), lds, stream, chains, r1, r2, F, dir);
    err = hipGetLastError();
  };
  if (dtype == EMRI_F32)
    ((K == Ks + 1 ? (one(std::integral_constant<int, Ks + 1>{}, type_tag<float>{}), true) : false) || ...);
  else
    ((K == Ks + 1 ? (one(std::integral_constant<int, Ks + 1>{}, type_tag<__half>{}), true) : false) || ...);
  return err;
}

template <int... Ks>
hipError_t launch_seed_move(int K, int max_seg, dim3 grid, hipStream_t stream, const ChainDesc *chains,
                            const float *draws, const double *f_init, int n_draw, float *cand, int64_t cand_stride,
                            std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  const size_t lds = stage_bytes(max_seg, K);
  auto one = [&](auto kc) {
    constexpr int KK = decltype(kc)::value;
    auto kern = lds ? seed_move_kernel<KK, true> : seed_move_kernel<KK, false>;
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return;
    hipLaunchKernelGGL(kern, grid, dim3(kSearchThreads), lds, stream, chains, draws, f_init, n_draw, cand,
                       cand_stride);
    err = hipGetLastError();
  };
  ((K == Ks + 1 ? (one(std::integral_constant<int, Ks + 1>{}), true) : false) || ...);
  return err;
}

using AllK = std::make_integer_sequence<int, EMRI_MAX_K>;

int check_chain(const emri_chain &c, int i) {
  if (c.n_walkers < 3) return fail(EMRI_EINVAL, "chain %d: n_walkers %d < 3", i, c.n_walkers);
  if (c.reserved != 0) return fail(EMRI_EINVAL, "chain %d: reserved must be zero", i);
  if (!c.f0 || !c.U || !c.box_lo || !c.box_hi || !c.coeffs || !c.stat)
    return fail(EMRI_EINVAL, "chain %d: a required pointer is NULL", i);
  const void *ptrs[] = {c.f0, c.U, c.box_lo, c.box_hi, c.coeffs, c.stat};
  for (const void *p : ptrs)
    if (!aligned16(p)) return fail(EMRI_EINVAL, "chain %d: device pointers must be 16-byte aligned", i);
  if (c.power.n_seg < 1) return fail(EMRI_EINVAL, "chain %d: no segments", i);
  return EMRI_OK;
}

struct SearchLayout {
  size_t chains, trials, total;
  std::vector<size_t> trial_off, tstat_off, pinv_off, popb_off, statb_off;
};

SearchLayout search_layout(const emri_chain *chains, int n, int K) {
  SearchLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes > 0 ? bytes : 1, 256);
    return at;
  };
  L.chains = take(sizeof(ChainDesc) * (size_t)n);
  L.trials = off;
  for (int i = 0; i < n; ++i) {
    L.trial_off.push_back(take(sizeof(float) * (size_t)chains[i].n_walkers * K));
    L.tstat_off.push_back(take(sizeof(float) * (size_t)chains[i].n_walkers));
    L.pinv_off.push_back(take(sizeof(double) * (size_t)chains[i].power.n_seg * K));
    L.popb_off.push_back(take(sizeof(float) * (size_t)chains[i].n_walkers * K));
    L.statb_off.push_back(take(sizeof(float) * (size_t)chains[i].n_walkers));
  }
  L.total = off;
  return L;
}

int validate_chains(const emri_chain *chains, int32_t n_chains, int32_t K) {
  if (!chains && n_chains > 0) return fail(EMRI_EINVAL, "chains is NULL");
  if (n_chains < 1 || n_chains > 65535) return fail(EMRI_EINVAL, "n_chains %d outside [1, 65535]", n_chains);
  if (K < 1 || K > EMRI_MAX_K) return fail(EMRI_EINVAL, "K = %d outside [1, %d]", K, EMRI_MAX_K);
  for (int i = 0; i < n_chains; ++i) {
    const int st = check_chain(chains[i], i);
    if (st) return st;
  }
  return EMRI_OK;
}

// What the trial kernel reads of a chain's spectrogram (the seeding scores
// through score_batched_plan, which checks the same).
int check_chain_power(const emri_chain &c, int i, int dtype) {
  const emri_power &pw = c.power;
  if (pw.dtype != EMRI_F32 && pw.dtype != EMRI_F16) return fail(EMRI_EINVAL, "chain %d: unknown power dtype", i);
  if (pw.dtype != dtype) return fail(EMRI_EINVAL, "chain %d: every chain must use the same power dtype", i);
  if (!pw.data || !aligned16(pw.data)) return fail(EMRI_EINVAL, "chain %d: power data NULL or not 16-byte aligned", i);
  if (pw.n_bins < 1 || pw.row_pitch < pw.n_bins || (pw.row_pitch % 8) != 0)
    return fail(EMRI_EINVAL, "chain %d: row_pitch must be a multiple of 8 and >= n_bins", i);
  if (!std::isfinite(pw.t_sft) || !(pw.t_sft > 0.0)) return fail(EMRI_EINVAL, "chain %d: bad t_sft", i);
  const int k_max = c.k_max < 0 ? pw.n_bins - 1 : c.k_max;
  if (c.k_min < 0 || k_max > pw.n_bins - 1 || c.k_min > k_max)
    return fail(EMRI_EINVAL, "chain %d: bin range outside the row", i);
  if ((uint64_t)pw.n_seg * (uint64_t)pw.row_pitch >= (1ull << 32))
    return fail(EMRI_EUNSUPPORTED, "chain %d: n_seg x row_pitch must stay below 2^32 elements", i);
  return EMRI_OK;
}

// Each chain's pseudo-inverse (transposed, n_seg x K) at dst + off[i]: its
// basis rows are copied to the host, inverted there and copied back.  Waits
// for the copies (set-up calls only).
int upload_pinv(const emri_chain *chains, int n, int K, char *dst, const std::vector<size_t> &off,
                hipStream_t stream) {
  std::vector<std::vector<double>> pt((size_t)n);
  std::vector<double> u;
  for (int i = 0; i < n; ++i) {
    const int ns = chains[i].power.n_seg;
    u.resize((size_t)ns * K);
    hipError_t err = hipMemcpyAsync(u.data(), chains[i].U, sizeof(double) * u.size(), hipMemcpyDeviceToHost, stream);
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "chain %d: basis copy: %s", i, hipGetErrorString(err));
    for (double v : u)
      if (!std::isfinite(v)) return fail(EMRI_EINVAL, "chain %d: the basis holds a non-finite value", i);
    pt[i].resize(u.size());
    pseudo_inverse_t(u.data(), ns, K, pt[i].data());
    err = hipMemcpyAsync(dst + off[i], pt[i].data(), sizeof(double) * pt[i].size(), hipMemcpyHostToDevice, stream);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "chain %d: pseudo-inverse copy: %s", i, hipGetErrorString(err));
  }
  const hipError_t err = hipStreamSynchronize(stream);      // pt holds the sources of the copies
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "pseudo-inverse copies: %s", hipGetErrorString(err));
  return EMRI_OK;
}

dim3 walker_grid(int max_walkers, int n_chains) {
  return dim3((unsigned)((max_walkers + kSearchThreads - 1) / kSearchThreads), (unsigned)n_chains);
}

}  // namespace

extern "C" int search_workspace_size(const emri_chain *chains, int32_t n_chains, int32_t K, size_t *bytes) {
  clear_error();
  if (!bytes) return fail(EMRI_EINVAL, "bytes is NULL");
  int st = validate_chains(chains, n_chains, K);
  if (st) return st;
  *bytes = search_layout(chains, n_chains, K).total;
  return EMRI_OK;
}

extern "C" int search_plan(const emri_chain *chains, int32_t n_chains, int32_t K, const batch_opts *opts,
                           void *workspace, size_t workspace_bytes, emri_search_plan *plan, void *hip_stream) {
  clear_error();
  if (!plan || !workspace) return fail(EMRI_EINVAL, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(EMRI_EINVAL, "workspace must be 256-byte aligned");
  int st = validate_chains(chains, n_chains, K);
  if (st) return st;
  if (opts) {
    for (int i = 0; i < 5; ++i)
      if (opts->reserved[i] != 0) return fail(EMRI_EINVAL, "batch_opts.reserved must be zero");
    if (opts->precision != EMRI_PLAIN)
      return fail(EMRI_EUNSUPPORTED, "generations score with FP64 positions (EMRI_PLAIN) only");
  }
  const int dtype = chains[0].power.dtype;
  for (int i = 0; i < n_chains; ++i)
    if ((st = check_chain_power(chains[i], i, dtype)) != EMRI_OK) return st;
  const SearchLayout L = search_layout(chains, n_chains, K);
  if (workspace_bytes < L.total)
    return fail(EMRI_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, L.total);
  char *ws = reinterpret_cast<char *>(workspace);
  std::vector<ChainDesc> desc((size_t)n_chains);
  int64_t offset = 0;
  int max_walkers = 0, max_seg = 0;
  for (int i = 0; i < n_chains; ++i) {
    ChainDesc &d = desc[i];
    std::memset(&d, 0, sizeof d);
    d.f0 = chains[i].f0;
    d.U = chains[i].U;
    d.box_lo = chains[i].box_lo;
    d.box_hi = chains[i].box_hi;
    d.coeffs = chains[i].coeffs;
    d.stat = chains[i].stat;
    d.pinvt = reinterpret_cast<const double *>(ws + L.pinv_off[i]);
    d.coeffs_b = reinterpret_cast<float *>(ws + L.popb_off[i]);
    d.stat_b = reinterpret_cast<float *>(ws + L.statb_off[i]);
    d.trial = reinterpret_cast<float *>(ws + L.trial_off[i]);
    d.trial_stat = reinterpret_cast<float *>(ws + L.tstat_off[i]);
    d.power = chains[i].power.data;
    d.t_sft = chains[i].power.t_sft;
    d.offset = offset;
    d.n_seg = chains[i].power.n_seg;
    d.n_walkers = chains[i].n_walkers;
    d.pitch = chains[i].power.row_pitch;
    d.k_min = chains[i].k_min;
    d.k_max = chains[i].k_max < 0 ? chains[i].power.n_bins - 1 : chains[i].k_max;
    offset += chains[i].n_walkers;
    max_walkers = std::max(max_walkers, chains[i].n_walkers);
    max_seg = std::max(max_seg, chains[i].power.n_seg);
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  if ((st = upload_pinv(chains, n_chains, K, ws, L.pinv_off, stream)) != EMRI_OK) return st;
  hipError_t err = hipMemcpyAsync(ws + L.chains, desc.data(), sizeof(ChainDesc) * desc.size(),
                                  hipMemcpyHostToDevice, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);     // desc is a host vector
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "search plan copy: %s", hipGetErrorString(err));
  SearchPlanData pd{};
  pd.magic = kSearchMagic;
  pd.n_chains = n_chains;
  pd.K = K;
  pd.max_walkers = max_walkers;
  pd.max_seg = max_seg;
  pd.dtype = dtype;
  pd.chains = reinterpret_cast<const ChainDesc *>(ws + L.chains);
  pd.total_walkers = offset;
  std::memset(plan, 0, sizeof *plan);
  std::memcpy(plan, &pd, sizeof pd);
  return EMRI_OK;
}

static int plan_data(const emri_search_plan *plan, SearchPlanData *pd) {
  if (!plan) return fail(EMRI_EINVAL, "plan is NULL");
  std::memcpy(pd, plan, sizeof *pd);
  if (pd->magic != kSearchMagic) return fail(EMRI_EINVAL, "plan was not made by search_plan");
  return EMRI_OK;
}

extern "C" int search_generation(const emri_search_plan *plan, const int32_t *r1, const int32_t *r2, const double *F,
                                 int32_t *accepted, void *hip_stream) {
  clear_error();
  SearchPlanData pd;
  int st = plan_data(plan, &pd);
  if (st) return st;
  if (!r1 || !r2 || !F) return fail(EMRI_EINVAL, "r1, r2 and F are required");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const dim3 sgrid((unsigned)((pd.max_walkers + kWalkersPerBlock - 1) / kWalkersPerBlock), (unsigned)pd.n_chains);
  hipError_t err = launch_trial_score(pd.K, pd.dtype, pd.max_seg, sgrid, stream, pd.chains, r1, r2, F, AllK{});
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "trial launch: %s", hipGetErrorString(err));
  hipLaunchKernelGGL(de_select_kernel, walker_grid(pd.max_walkers, pd.n_chains), dim3(kSearchThreads), 0, stream,
                     pd.chains, pd.K, accepted);
  err = hipGetLastError();
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "select launch: %s", hipGetErrorString(err));
  return EMRI_OK;
}

extern "C" int search_generations(const emri_search_plan *plan, int32_t n_gen, const int32_t *r1, const int32_t *r2,
                                  const double *F, void *hip_stream) {
  clear_error();
  SearchPlanData pd;
  int st = plan_data(plan, &pd);
  if (st) return st;
  if (n_gen < 0) return fail(EMRI_EINVAL, "n_gen %d < 0", n_gen);
  if (n_gen > 0 && (!r1 || !r2 || !F)) return fail(EMRI_EINVAL, "r1, r2 and F are required");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const dim3 sgrid((unsigned)((pd.max_walkers + kWalkersPerBlock - 1) / kWalkersPerBlock), (unsigned)pd.n_chains);
  const int64_t T = pd.total_walkers;
  int g = 0;
  for (; g + 1 < n_gen; g += 2) {       // a pair: to the workspace copy and back, one launch each
    for (int dir = 0; dir < 2; ++dir) {
      const int64_t o = (int64_t)(g + dir) * T;
      hipError_t err = launch_generation(pd.K, pd.dtype, pd.max_seg, sgrid, stream, pd.chains, r1 + o, r2 + o, F + o,
                                         dir, AllK{});
      if (err != hipSuccess) return fail(EMRI_EDEVICE, "generation launch: %s", hipGetErrorString(err));
    }
  }
  if (g < n_gen) {                      // an odd last generation: trials, then selection in place
    const int64_t o = (int64_t)g * T;
    hipError_t err = launch_trial_score(pd.K, pd.dtype, pd.max_seg, sgrid, stream, pd.chains, r1 + o, r2 + o, F + o,
                                        AllK{});
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "trial launch: %s", hipGetErrorString(err));
    hipLaunchKernelGGL(de_select_kernel, walker_grid(pd.max_walkers, pd.n_chains), dim3(kSearchThreads), 0, stream,
                       pd.chains, pd.K, nullptr);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "select launch: %s", hipGetErrorString(err));
  }
  return EMRI_OK;
}

extern "C" int search_best(const emri_search_plan *plan, const double *noise_mean, const double *noise_std,
                           float *best_stat, int32_t *best_idx, double *best_norm, void *hip_stream) {
  clear_error();
  SearchPlanData pd;
  int st = plan_data(plan, &pd);
  if (st) return st;
  if (!best_stat || !best_idx) return fail(EMRI_EINVAL, "best_stat and best_idx are required");
  if (best_norm && (!noise_mean || !noise_std)) return fail(EMRI_EINVAL, "best_norm needs noise_mean and noise_std");
  hipLaunchKernelGGL(search_best_kernel, dim3(pd.n_chains), dim3(kSearchThreads), 0,
                     reinterpret_cast<hipStream_t>(hip_stream), pd.chains, noise_mean, noise_std, best_stat, best_idx,
                     best_norm);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "best launch: %s", hipGetErrorString(err));
  return EMRI_OK;
}

extern "C" int search_noise_moments(const float *best, int32_t n_real, int32_t n_chains, double *mean, double *sd,
                                    void *hip_stream) {
  clear_error();
  if (!best || !mean || !sd) return fail(EMRI_EINVAL, "NULL argument");
  if (n_real < 2 || n_chains < 1) return fail(EMRI_EINVAL, "need n_real >= 2 and n_chains >= 1");
  hipLaunchKernelGGL(noise_moments_kernel, dim3((unsigned)((n_chains + kSearchThreads - 1) / kSearchThreads)),
                     dim3(kSearchThreads), 0, reinterpret_cast<hipStream_t>(hip_stream), best, n_real, n_chains, mean,
                     sd);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "moments launch: %s", hipGetErrorString(err));
  return EMRI_OK;
}

namespace {

// Per chain, at 256-byte strides: candidates (n_draw x K FP32), their
// statistics, the top-n_walkers values and indices; then the chain table and
// the candidates' scoring workspace.
struct SeedLayout {
  int64_t cand_stride, stat_stride, top_stride;     // elements per chain
  size_t cand, stat, top_val, top_idx, table, scoring, total;
  std::vector<size_t> pinv_off;
};

SeedLayout seed_layout(const emri_chain *chains, int n_chains, int n_draw, int max_walkers, int K,
                       size_t scoring_bytes) {
  SeedLayout L;
  L.cand_stride = (int64_t)round_up((size_t)n_draw * K, 64);
  L.stat_stride = (int64_t)round_up((size_t)n_draw, 64);
  L.top_stride = (int64_t)round_up((size_t)max_walkers, 64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes > 0 ? bytes : 1, 256);
    return at;
  };
  L.cand = take(sizeof(float) * (size_t)n_chains * L.cand_stride);
  L.stat = take(sizeof(float) * (size_t)n_chains * L.stat_stride);
  L.top_val = take(sizeof(float) * (size_t)n_chains * L.top_stride);
  L.top_idx = take(sizeof(int64_t) * (size_t)n_chains * L.top_stride);
  L.table = take(sizeof(ChainDesc) * (size_t)n_chains);
  for (int i = 0; i < n_chains; ++i) L.pinv_off.push_back(take(sizeof(double) * (size_t)chains[i].power.n_seg * K));
  L.scoring = take(scoring_bytes);
  L.total = off;
  return L;
}

// Candidate problems of the seeding: chain i's n_draw candidates, top n_walkers.
std::vector<emri_problem> seed_problems(const emri_chain *chains, int n, int n_draw, char *ws, const SeedLayout &L) {
  std::vector<emri_problem> pbs((size_t)n);
  // sizing calls pass no workspace: any aligned non-null address stands in
  char *base = ws ? ws : reinterpret_cast<char *>(256);
  for (int i = 0; i < n; ++i) {
    emri_problem &p = pbs[i];
    std::memset(&p, 0, sizeof p);
    p.power = chains[i].power;
    p.f0 = chains[i].f0;
    p.U = chains[i].U;
    p.coeffs = reinterpret_cast<const float *>(base + L.cand + sizeof(float) * (size_t)i * L.cand_stride);
    p.n_tmpl = n_draw;
    p.top_k = chains[i].n_walkers;
    p.k_min = chains[i].k_min;
    p.k_max = chains[i].k_max;
    p.stat = reinterpret_cast<float *>(base + L.stat + sizeof(float) * (size_t)i * L.stat_stride);
    p.topk_val = reinterpret_cast<float *>(base + L.top_val + sizeof(float) * (size_t)i * L.top_stride);
    p.topk_idx = reinterpret_cast<int64_t *>(base + L.top_idx + sizeof(int64_t) * (size_t)i * L.top_stride);
  }
  return pbs;
}

int seed_sizes(const emri_chain *chains, int32_t n_chains, int32_t K, int32_t n_draw, int *max_walkers,
               size_t *scoring) {
  int st = validate_chains(chains, n_chains, K);
  if (st) return st;
  if (n_draw < 1 || n_draw > (1 << 28)) return fail(EMRI_EINVAL, "n_draw %d out of range", n_draw);
  *max_walkers = 0;
  for (int i = 0; i < n_chains; ++i) {
    if (chains[i].n_walkers > n_draw)
      return fail(EMRI_EINVAL, "chain %d keeps %d walkers of only %d candidates", i, chains[i].n_walkers, n_draw);
    if (chains[i].n_walkers > EMRI_MAX_TOPK)
      return fail(EMRI_EUNSUPPORTED, "chain %d: seeding keeps at most %d walkers", i, EMRI_MAX_TOPK);
    *max_walkers = std::max(*max_walkers, chains[i].n_walkers);
  }
  const SeedLayout L0 = seed_layout(chains, n_chains, n_draw, *max_walkers, K, 0);
  std::vector<emri_problem> pbs = seed_problems(chains, n_chains, n_draw, nullptr, L0);
  return score_batched_workspace_size(pbs.data(), n_chains, K, scoring);
}

}  // namespace

extern "C" int search_seed_workspace_size(const emri_chain *chains, int32_t n_chains, int32_t K, int32_t n_draw,
                                          size_t *bytes) {
  clear_error();
  if (!bytes) return fail(EMRI_EINVAL, "bytes is NULL");
  int mw = 0;
  size_t sb = 0;
  const int st = seed_sizes(chains, n_chains, K, n_draw, &mw, &sb);
  if (st) return st;
  *bytes = seed_layout(chains, n_chains, n_draw, mw, K, sb).total;
  return EMRI_OK;
}

extern "C" int search_seed(const emri_chain *chains, int32_t n_chains, int32_t K, const float *draws,
                           const double *f_init, int32_t n_draw, const batch_opts *opts, void *workspace,
                           size_t workspace_bytes, void *hip_stream) {
  clear_error();
  if (!workspace || !draws || !f_init) return fail(EMRI_EINVAL, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(EMRI_EINVAL, "workspace must be 256-byte aligned");
  if (!aligned16(draws) || !aligned16(f_init)) return fail(EMRI_EINVAL, "device pointers must be 16-byte aligned");
  int mw = 0;
  size_t sb = 0;
  int st = seed_sizes(chains, n_chains, K, n_draw, &mw, &sb);
  if (st) return st;
  const SeedLayout L = seed_layout(chains, n_chains, n_draw, mw, K, sb);
  if (workspace_bytes < L.total)
    return fail(EMRI_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, L.total);
  char *ws = reinterpret_cast<char *>(workspace);
  std::vector<ChainDesc> desc((size_t)n_chains);
  for (int i = 0; i < n_chains; ++i) {
    std::memset(&desc[i], 0, sizeof desc[i]);
    desc[i].f0 = chains[i].f0;
    desc[i].U = chains[i].U;
    desc[i].pinvt = reinterpret_cast<const double *>(ws + L.pinv_off[i]);
    desc[i].coeffs = chains[i].coeffs;
    desc[i].stat = chains[i].stat;
    desc[i].n_seg = chains[i].power.n_seg;
    desc[i].n_walkers = chains[i].n_walkers;
  }
  std::vector<emri_problem> pbs = seed_problems(chains, n_chains, n_draw, ws, L);
  emri_batch_plan scoring;
  if ((st = score_batched_plan(pbs.data(), n_chains, K, opts, ws + L.scoring, workspace_bytes - L.scoring, &scoring,
                               hip_stream)) != EMRI_OK)
    return st;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  ChainDesc *d_desc = reinterpret_cast<ChainDesc *>(ws + L.table);
  if ((st = upload_pinv(chains, n_chains, K, ws, L.pinv_off, stream)) != EMRI_OK) return st;
  hipError_t err = hipMemcpyAsync(d_desc, desc.data(), sizeof(ChainDesc) * desc.size(), hipMemcpyHostToDevice, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);      // desc is a host vector
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "seed table copy: %s", hipGetErrorString(err));
  float *cand = reinterpret_cast<float *>(ws + L.cand);
  int max_seg = 0;
  for (int i = 0; i < n_chains; ++i) max_seg = std::max(max_seg, chains[i].power.n_seg);
  err = launch_seed_move(K, max_seg, walker_grid(n_draw, n_chains), stream, d_desc, draws, f_init, n_draw, cand,
                         L.cand_stride, AllK{});
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "seed launch: %s", hipGetErrorString(err));
  if ((st = score_batched_run(&scoring, hip_stream)) != EMRI_OK) return st;
  hipLaunchKernelGGL(seed_gather_kernel, walker_grid(mw, n_chains), dim3(kSearchThreads), 0, stream, d_desc, K, cand,
                     L.cand_stride, reinterpret_cast<const float *>(ws + L.top_val),
                     reinterpret_cast<const int64_t *>(ws + L.top_idx), L.top_stride);
  if ((err = hipGetLastError()) != hipSuccess) return fail(EMRI_EDEVICE, "seed gather: %s", hipGetErrorString(err));
  return EMRI_OK;
}
