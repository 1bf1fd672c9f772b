// Re-scoring of selected templates with FP64 positions, and the final top-k
// of the re-scored candidates.
//
// The mixed-precision form rounds FP32-accumulated positions, so a position
// that lies within the FP32 error of a half-integer can land in the
// neighbouring bin (Eq. (6) then sums a different power for that segment).
// With rescore_top set, score_tracks takes the best `kc` templates of the
// mixed statistic, evaluates each of them again exactly as the plain path
// does (FP64 fused multiply-adds in k order from f0 T, round half to even,
// FP32 runs of 8 segments summed in FP64 in segment order), writes those
// statistics into stat, and orders the candidates by (-S, index) for the
// top-k.  The re-scored statistic equals the plain path's bit for bit.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "common.h"
#include "rescore_internal.h"
#include "topk_device.h"

namespace emri {
namespace {

constexpr double kWild = 67108864.0;          // 2^26 bins: positions beyond contribute nothing
constexpr int RESCORE_WAVES = 4;              // candidates per workgroup (one wave each)
constexpr int SELECT_THREADS = 1024;

template <typename PT>
__device__ __forceinline__ float power_at(const void *data, int64_t off) {
  if constexpr (sizeof(PT) == 4) {
    return reinterpret_cast<const float *>(data)[off];
  } else {
    return (float)__builtin_bit_cast(_Float16, reinterpret_cast<const unsigned short *>(data)[off]);
  }
}

// One wave per candidate.  Lane l evaluates segments base + 8l .. base + 8l + 7
// of each chunk of 512, which is exactly one run of the plain kernel's FP32
// accumulation; the runs are then added into the FP64 sum in segment order.
template <typename PT>
__global__ __launch_bounds__(64 * RESCORE_WAVES) void rescore_kernel(RescoreParams r) {
  const int lane = (int)(threadIdx.x & 63);
  const int c = (int)blockIdx.x * RESCORE_WAVES + (int)(threadIdx.x >> 6);
  if (c >= r.n_cand) return;                 // whole waves leave together
  const int64_t j = r.cand_idx[c];
  if (j < 0 || j >= r.n_tmpl) return;
  double cd[EMRI_MAX_K];
#pragma unroll
  for (int k = 0; k < EMRI_MAX_K; ++k) cd[k] = k < r.K ? (double)r.coeffs[(size_t)j * r.K + k] : 0.0;
  double sum = 0.0;
  for (int base = 0; base < r.n_seg; base += 512) {
    float acc = 0.0f;
    for (int i = 0; i < 8; ++i) {
      const int a = base + 8 * lane + i;
      if (a < r.n_seg) {
        const double *sc = r.seg + (size_t)a * r.seg_stride;
        double y = sc[0];
#pragma unroll
        for (int k = 0; k < EMRI_MAX_K; ++k)
          if (k < r.K) y = __builtin_fma(cd[k], sc[1 + k], y);
        float v = 0.0f;
        if (__builtin_fabs(y) < kWild) {
          const double b = __builtin_rint(y);          // half to even
          if (b >= (double)r.k_min && b <= (double)r.k_max)
            v = power_at<PT>(r.power, (int64_t)a * r.row_pitch + (int64_t)b);
        }
        acc = acc + v;
      }
    }
    // runs of this chunk in segment order (lane l holds run base/8 + l)
    for (int l = 0; l < 64 && base + 8 * l < r.n_seg; ++l) sum += (double)__shfl(acc, l, 64);
  }
  if (lane == 0) {
    r.stat[j] = (float)sum;
    r.cand_val[c] = (float)sum;
  }
}

// One workgroup: the rank of every candidate under (-S, index) by counting
// the candidates ahead of it (the keys are distinct, so ranks are a
// permutation); ranks below top_k are written out, and positions past the
// candidates are padded with (-inf, -1).
__global__ __launch_bounds__(SELECT_THREADS) void rescore_select_kernel(const float *cand_val,
                                                                        const int64_t *cand_idx, int n_cand,
                                                                        int top_k, float *out_val,
                                                                        int64_t *out_idx) {
  __shared__ unsigned long long keys[RESCORE_MAX_CAND];
  for (int i = threadIdx.x; i < n_cand; i += SELECT_THREADS) {
    const uint32_t idx = (uint32_t)cand_idx[i];
    keys[i] = ((unsigned long long)order_key(cand_val[i]) << 32) | (unsigned long long)(0xffffffffu - idx);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_cand; i += SELECT_THREADS) {
    const unsigned long long ki = keys[i];
    int rank = 0;
    for (int m = 0; m < n_cand; ++m) rank += keys[m] > ki ? 1 : 0;
    if (rank < top_k) {
      out_val[rank] = cand_val[i];
      out_idx[rank] = cand_idx[i];
    }
  }
  for (int i = n_cand + (int)threadIdx.x; i < top_k; i += SELECT_THREADS) {
    out_val[i] = -__builtin_inff();
    out_idx[i] = -1;
  }
}

}  // namespace

int rescore_candidates(int top_k, int64_t n_tmpl) {
  int64_t kc = 4 * (int64_t)top_k;
  if (kc < 64) kc = 64;
  if (kc > RESCORE_MAX_CAND) kc = RESCORE_MAX_CAND;
  if (kc < top_k) kc = top_k;
  return (int)(kc < n_tmpl ? kc : n_tmpl);
}

hipError_t launch_rescore(const RescoreParams &r, int dtype, hipStream_t stream) {
  if (r.n_cand <= 0) return hipSuccess;
  const int grid = (r.n_cand + RESCORE_WAVES - 1) / RESCORE_WAVES;
  if (dtype == EMRI_F32)
    hipLaunchKernelGGL(rescore_kernel<float>, dim3(grid), dim3(64 * RESCORE_WAVES), 0, stream, r);
  else
    hipLaunchKernelGGL(rescore_kernel<__half>, dim3(grid), dim3(64 * RESCORE_WAVES), 0, stream, r);
  return hipGetLastError();
}

hipError_t launch_rescore_select(const float *cand_val, const int64_t *cand_idx, int n_cand, int top_k,
                                 float *out_val, int64_t *out_idx, hipStream_t stream) {
  if (top_k <= 0) return hipSuccess;
  hipLaunchKernelGGL(rescore_select_kernel, dim3(1), dim3(SELECT_THREADS), 0, stream, cand_val, cand_idx, n_cand,
                     top_k, out_val, out_idx);
  return hipGetLastError();
}

}  // namespace emri
