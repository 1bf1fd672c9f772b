// build_sfts: Hann-windowed real DFT of every SFT segment and PSD normalisation
// (Sec. II B segments of duration T_SFT with bin width 1/T_SFT; Eq. (7) weights
// each bin by 1/S_n(f); Sec. II F takes the PSD as known).
//
// One workgroup per segment.  The N real samples are packed into N/2 complex
// values z_m = w_{2m} x_{2m} + i w_{2m+1} x_{2m+1}, transformed with a
// mixed-radix (2, 3, 4, 5, 7) Stockham FFT held entirely in LDS in FP64
// (N/2 * 16 B <= 160 KB), and split into the real DFT
//   X_b = E_b + e^{-2 pi i b / N} O_b,
//   E_b = (Z_b + conj Z_{M-b}) / 2,  O_b = (Z_b - conj Z_{M-b}) / (2i).
// Each radix pass reads its butterfly inputs into registers, synchronises, then
// writes its outputs in place, so a single LDS buffer suffices.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "common.h"

namespace emri {
namespace {

constexpr int SFT_THREADS = 1024;
constexpr int SFT_MAX_M = 10240;        // N/2 complex values in 160 KB of LDS
constexpr int SFT_MAX_STAGES = 24;

struct SftPlan {
  int M;                      // N/2
  int n_stages;
  int radix[SFT_MAX_STAGES];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-register DFT of length R (forward, e^{-2 pi i r q / R}).
template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R]) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
  } else if constexpr (R == 4) {
    const double2 s02 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
    const double2 d02 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
    const double2 s13 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
    const double2 d13 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
    v[0] = make_double2(s02.x + s13.x, s02.y + s13.y);
    v[2] = make_double2(s02.x - s13.x, s02.y - s13.y);
    // -i * d13 = (d13.y, -d13.x)
    v[1] = make_double2(d02.x + d13.y, d02.y - d13.x);
    v[3] = make_double2(d02.x - d13.y, d02.y + d13.x);
  } else if constexpr (R == 3) {
    const double s3 = 0.86602540378443864676;   // sin(2 pi / 3)
    const double2 t = make_double2(v[1].x + v[2].x, v[1].y + v[2].y);
    const double2 d = make_double2(v[1].x - v[2].x, v[1].y - v[2].y);
    const double2 m = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    v[0] = make_double2(v[0].x + t.x, v[0].y + t.y);
    // V1 = m - i s d ; V2 = m + i s d  (i d = (-d.y, d.x))
    v[1] = make_double2(m.x + s3 * d.y, m.y - s3 * d.x);
    v[2] = make_double2(m.x - s3 * d.y, m.y + s3 * d.x);
  } else {
    double2 w[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      double s, c;
      sincospi(-2.0 * m / R, &s, &c);
      w[m] = make_double2(c, s);
    }
    double2 out[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double2 acc = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const double2 p = cmul(v[r], w[(r * q) % R]);
        acc.x += p.x;
        acc.y += p.y;
      }
      out[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = out[q];
  }
}

// One Stockham pass of radix R over M points with Ns = product of earlier radices.
template <int R>
__device__ void stockham_pass(double2 *z, int M, int Ns) {
  constexpr int BMAX = (SFT_MAX_M + R * SFT_THREADS - 1) / (R * SFT_THREADS);
  const int nb = M / R;
  double2 v[BMAX][R];
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int j = threadIdx.x + i * SFT_THREADS;
    if (j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = z[j + r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int j = threadIdx.x + i * SFT_THREADS;
    if (j < nb) {
      const int k = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double s, c;
          sincospi(-2.0 * (double)(k * r) / (double)(Ns * R), &s, &c);
          v[i][r] = cmul(v[i][r], make_double2(c, s));
        }
      }
      small_dft<R>(v[i]);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) z[base + q * Ns] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename PT>
__device__ __forceinline__ PT to_storage(double v);
template <>
__device__ __forceinline__ float to_storage<float>(double v) { return (float)v; }
// FP64 -> FP16 with a single rounding: round to odd at FP32 precision (24 bits,
// at least two more than FP16 carries), then round to nearest-even FP16.
template <>
__device__ __forceinline__ __half to_storage<__half>(double v) {
  float f = (float)v;
  // one step toward zero: the magnitude bits drop by one ulp (inf becomes FLT_MAX)
  if (__builtin_fabs((double)f) > __builtin_fabs(v)) f = __uint_as_float(__float_as_uint(f) - 1u);
  if ((double)f != v && v == v) f = __uint_as_float(__float_as_uint(f) | 1u);
  return __float2half(f);
}

// Power output (FP32 or FP16 element per bin), or with PT = float2 the whitened
// complex SFT X_b / sqrt(sum w^2 S_b / (2 dt)) as (re, im) FP32 pairs.
template <typename PT>
__device__ __forceinline__ PT sft_store(double xr, double xi, double scale2);
template <>
__device__ __forceinline__ float sft_store<float>(double xr, double xi, double scale2) {
  return to_storage<float>((xr * xr + xi * xi) * scale2);
}
template <>
__device__ __forceinline__ __half sft_store<__half>(double xr, double xi, double scale2) {
  return to_storage<__half>((xr * xr + xi * xi) * scale2);
}
template <>
__device__ __forceinline__ float2 sft_store<float2>(double xr, double xi, double scale2) {
  const double s = __builtin_sqrt(scale2);
  return make_float2((float)(xr * s), (float)(xi * s));
}
template <typename PT>
__device__ __forceinline__ PT sft_zero();
template <>
__device__ __forceinline__ float sft_zero<float>() { return 0.0f; }
template <>
__device__ __forceinline__ __half sft_zero<__half>() { return to_storage<__half>(0.0); }
template <>
__device__ __forceinline__ float2 sft_zero<float2>() { return make_float2(0.0f, 0.0f); }

template <typename PT>
__global__ __launch_bounds__(SFT_THREADS) void sft_kernel(const double *__restrict__ x, int n_sft, double dt,
                                                           const double *__restrict__ psd, PT *__restrict__ out,
                                                           int row_pitch, SftPlan plan) {
  extern __shared__ double2 z[];
  const int M = plan.M;
  const int N = n_sft;
  const double *seg = x + (size_t)blockIdx.x * (size_t)N;
  for (int m = threadIdx.x; m < M; m += SFT_THREADS) {
    const double2 p = reinterpret_cast<const double2 *>(seg)[m];
    const double w0 = sinpi((double)(2 * m) / N);
    const double w1 = sinpi((double)(2 * m + 1) / N);
    z[m] = make_double2(w0 * w0 * p.x, w1 * w1 * p.y);
  }
  __syncthreads();
  int Ns = 1;
  for (int st = 0; st < plan.n_stages; ++st) {
    const int R = plan.radix[st];
    switch (R) {
      case 4: stockham_pass<4>(z, M, Ns); break;
      case 2: stockham_pass<2>(z, M, Ns); break;
      case 3: stockham_pass<3>(z, M, Ns); break;
      case 5: stockham_pass<5>(z, M, Ns); break;
      default: stockham_pass<7>(z, M, Ns); break;
    }
    Ns *= R;
  }
  // real-DFT split, normalisation and store (the row is written once, coalesced)
  const double sum_w2 = 0.375 * (double)N;
  PT *row = out + (size_t)blockIdx.x * (size_t)row_pitch;
  for (int b = threadIdx.x; b < row_pitch; b += SFT_THREADS) {
    PT p = sft_zero<PT>();
    if (b <= M) {
      const double s_b = psd[b];
      if (s_b > 0.0 && s_b <= 1.7976931348623157e308) {
        const double2 zb = z[b == M ? 0 : b];
        const double2 zc = z[b == 0 ? 0 : M - b];      // Z_{M-b}, with Z_M = Z_0
        const double2 e = make_double2(0.5 * (zb.x + zc.x), 0.5 * (zb.y - zc.y));
        // (Z_b - conj Z_{M-b}) / (2i)
        const double2 d = make_double2(zb.x - zc.x, zb.y + zc.y);
        const double2 o = make_double2(0.5 * d.y, -0.5 * d.x);
        double s, c;
        sincospi(-(double)b / (double)M, &s, &c);
        const double2 t = cmul(o, make_double2(c, s));
        const double xr = e.x + t.x, xi = e.y + t.y;
        p = sft_store<PT>(xr, xi, (2.0 * dt) / (sum_w2 * s_b));
      }
    }
    row[b] = p;
  }
}

bool make_plan(int M, SftPlan *plan) {
  plan->M = M;
  plan->n_stages = 0;
  int m = M;
  auto push = [&](int r) {
    if (plan->n_stages >= SFT_MAX_STAGES) return false;
    plan->radix[plan->n_stages++] = r;
    return true;
  };
  while (m % 4 == 0) { if (!push(4)) return false; m /= 4; }
  for (int p : {2, 3, 5, 7})
    while (m % p == 0) { if (!push(p)) return false; m /= p; }
  return m == 1;
}

}  // namespace
}  // namespace emri

using namespace emri;

extern "C" int build_sfts(const double *x, int64_t n_samples, double dt, int32_t n_sft, const double *psd,
                          emri_power *out, void *hip_stream) {
  clear_error();
  if (!out) return fail(EMRI_EINVAL, "out is NULL");
  if (!x || !psd) return fail(EMRI_EINVAL, "x or psd is NULL");
  if (n_samples < 0) return fail(EMRI_EINVAL, "n_samples < 0");
  if (!(dt > 0.0) || !(dt < 1e300)) return fail(EMRI_EINVAL, "dt must be finite and > 0");
  if (n_sft < 4 || (n_sft & 1)) return fail(EMRI_EINVAL, "n_sft must be even and >= 4");
  if (out->dtype != EMRI_F32 && out->dtype != EMRI_F16 && out->dtype != EMRI_C32)
    return fail(EMRI_EINVAL, "unknown power dtype %d", out->dtype);
  const int n_bins = n_sft / 2 + 1;
  if (out->row_pitch < n_bins || (out->row_pitch % 8) != 0)
    return fail(EMRI_EINVAL, "row_pitch %d must be a multiple of 8 and >= n_bins %d", out->row_pitch, n_bins);
  if (!aligned16(x) || !aligned16(psd) || !aligned16(out->data))
    return fail(EMRI_EINVAL, "device pointers must be 16-byte aligned");
  const int M = n_sft / 2;
  SftPlan plan;
  if (M > SFT_MAX_M) return fail(EMRI_EUNSUPPORTED, "n_sft %d exceeds %d", n_sft, 2 * SFT_MAX_M);
  if (!make_plan(M, &plan)) return fail(EMRI_EUNSUPPORTED, "n_sft/2 = %d has a prime factor above 7", M);
  const int64_t n_seg = n_samples / n_sft;
  if (n_seg > INT32_MAX) return fail(EMRI_ERANGE, "too many segments");
  if (n_seg > 0 && !out->data) return fail(EMRI_EINVAL, "out->data is NULL");
  out->n_seg = (int32_t)n_seg;
  out->n_bins = n_bins;
  out->t_sft = (double)n_sft * dt;
  if (n_seg == 0) return EMRI_OK;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t lds = (size_t)M * sizeof(double2);
  hipError_t err;
  if (out->dtype == EMRI_F32) {
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(&sft_kernel<float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(sft_kernel<float>, dim3((unsigned)n_seg), dim3(SFT_THREADS), lds, stream, x, n_sft, dt,
                         psd, reinterpret_cast<float *>(out->data), out->row_pitch, plan);
      err = hipGetLastError();
    }
  } else if (out->dtype == EMRI_C32) {
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(&sft_kernel<float2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(sft_kernel<float2>, dim3((unsigned)n_seg), dim3(SFT_THREADS), lds, stream, x, n_sft, dt,
                         psd, reinterpret_cast<float2 *>(out->data), out->row_pitch, plan);
      err = hipGetLastError();
    }
  } else {
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(&sft_kernel<__half>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(sft_kernel<__half>, dim3((unsigned)n_seg), dim3(SFT_THREADS), lds, stream, x, n_sft, dt,
                         psd, reinterpret_cast<__half *>(out->data), out->row_pitch, plan);
      err = hipGetLastError();
    }
  }
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "build_sfts launch: %s", hipGetErrorString(err));
  return EMRI_OK;
}
