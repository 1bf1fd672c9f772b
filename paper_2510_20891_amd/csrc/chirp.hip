// The linear-chirp statistic (Sec. II B, Eqs. (4)-(7)): every segment's
// signal is a chirping sinusoid with the track's local frequency f and
// derivative fdot, its template SFT is evaluated over the 2P + 1 bins around
// rint(f T), and the phase- and amplitude-maximised inner product with the
// whitened data SFT is summed over the segments that pass the validity cut
// (|fddot| T^3 / 6 <= 1) and the cut-offs of Sec. II D.
//
// Per template (one wave) and segment:
//   * the track f[alpha] = f0 + sum_k c_k U[alpha, k] (FP64) is built once per
//     template in LDS; fdot and fddot are second-order finite differences
//     (central inside, one-sided at the ends for fdot, the neighbour's fddot
//     at the ends);
//   * the template SFT of the unit chirp, Hann-windowed,
//         H_{k0 + j} ~ R(d0 - j, b),  R(d, b) = int cos^2(pi u) e^{2 pi i d u + i pi b u^2} du,
//     d0 = f T - k0, b = fdot T^2, is the M = 256-point DFT of its samples
//     g_m = sin^2(pi m / M) e^{i pi (b u^2 + 2 d0 u)}, u = m / M - 1/2 (up to a
//     common factor; the integrand vanishes smoothly at both ends, so the
//     sum converges like the integral's aliased tail: relative error below
//     4e-7 for |b| <= 60 and P = 100), by a four-pass radix-4 Stockham FFT in
//     the wave's LDS (one butterfly per lane per pass), FP32;
//   * S_alpha = |sum_k conj(Z_k) H_k / sqrt(S_k)|^2 / sum_k |H_k|^2 / S_k over
//     the window's bins inside the row (FP32 products, FP64 cross-lane sums),
//     0 when the central bin rint(f T) is outside the row;
//   * S = sum of S_alpha over valid segments, FP64, stored FP32.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "score_internal.h"
#include "topk_internal.h"
#include "topk_device.h"

namespace emri {
namespace {

constexpr int CH_M = 256;            // template samples (FFT length)
constexpr int CH_QUARTER = CH_M / 4; // butterflies per radix-4 pass = lanes of a wave
constexpr int CH_WAVES = 4;          // templates per workgroup
constexpr int CH_THREADS = 64 * CH_WAVES;
constexpr int CH_MAX_P = 100;        // 2P + 1 <= 201 bins
constexpr int CH_MAX_SEG = 2048;     // track of every wave's template in LDS
constexpr int CH_WIN = 2 * CH_MAX_P + 1;
static_assert(CH_QUARTER == 64, "one butterfly per lane");
static_assert((CH_WIN + 63) / 64 <= 4, "window bins per lane");

struct ChirpParams {
  const float2 *Z;            // n_seg rows x pitch bins
  const float *isq;           // 1/sqrt(S_k), 0 for bins without a usable PSD
  const double *f0, *U;       // track basis
  const float *coeffs;        // n_tmpl x K
  float *stat;
  int64_t n_tmpl;
  double t_sft, f_min, fdot_min;
  int pitch, n_seg, n_bins, K;
  int p_half, pad;
};

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ void lds_wave_sync() {
  // the wave's LDS writes are complete before any lane reads another lane's data
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Forward DFT of the wave's 256 samples in src (result in src after four
// passes that alternate src / dst); tw[m] = e^{-2 pi i m / 256}.
__device__ __forceinline__ float2 *fft256(float2 *src, float2 *dst, const float2 *tw, int lane) {
  int Ns = 1;
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int k = lane % Ns;
    float2 v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float2 x = src[lane + r * CH_QUARTER];
      v[r] = r == 0 ? x : cmulf(x, tw[(r * k * (CH_M / (4 * Ns))) & (CH_M - 1)]);
    }
    const float2 s02 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
    const float2 d02 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
    const float2 s13 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
    const float2 d13 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
    const int base = (lane / Ns) * 4 * Ns + k;
    dst[base] = make_float2(s02.x + s13.x, s02.y + s13.y);
    dst[base + Ns] = make_float2(d02.x + d13.y, d02.y - d13.x);          // a - i b - c + i d
    dst[base + 2 * Ns] = make_float2(s02.x - s13.x, s02.y - s13.y);
    dst[base + 3 * Ns] = make_float2(d02.x - d13.y, d02.y + d13.x);      // a + i b - c - i d
    lds_wave_sync();
    float2 *t = src;
    src = dst;
    dst = t;
    Ns *= 4;
  }
  return src;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int CH_RESET_PARTS = 8;

// 1/sqrt(S_k) per bin; workgroups past the bins' clear the top-k state of the
// call, a share each.
__global__ __launch_bounds__(CH_THREADS) void chirp_prep_kernel(const double *__restrict__ psd, int n_bins,
                                                                float *__restrict__ isq, TopkState *topk) {
  const int bin_blocks = (n_bins + CH_THREADS - 1) / CH_THREADS;
  if ((int)blockIdx.x >= bin_blocks) {
    topk_state_reset(topk, (int)blockIdx.x - bin_blocks, CH_RESET_PARTS);
    return;
  }
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_bins) return;
  const double s = psd[k];
  isq[k] = (s > 0.0 && s <= 1.7976931348623157e308) ? (float)(1.0 / __builtin_sqrt(s)) : 0.0f;
}

__global__ __launch_bounds__(CH_THREADS) void chirp_score_kernel(ChirpParams p) {
  __shared__ float2 tw[CH_M];
  __shared__ float win[CH_M];
  __shared__ float2 buf[CH_WAVES][2][CH_M];
  extern __shared__ double track_lds[];
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  for (int m = threadIdx.x; m < CH_M; m += CH_THREADS) {
    double s, c;
    sincospi(-2.0 * (double)m / CH_M, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
    const double w = sinpi((double)m / CH_M);
    win[m] = (float)(w * w);
  }
  const int64_t j = (int64_t)blockIdx.x * CH_WAVES + wave;
  const bool live = j < p.n_tmpl;
  double *track = track_lds + (size_t)wave * p.n_seg;
  if (live) {
    for (int a = lane; a < p.n_seg; a += 64) {
      double f = p.f0[a];
      for (int k = 0; k < p.K; ++k) f = __builtin_fma((double)p.coeffs[(size_t)j * p.K + k], p.U[(size_t)a * p.K + k], f);
      track[a] = f;
    }
  }
  __syncthreads();                     // tables and tracks; no block-wide barrier follows
  if (!live) return;
  const double T = p.t_sft;
  const int n = p.n_seg;
  double total = 0.0;
  for (int a = 0; a < n; ++a) {
    // local frequency and its derivatives (wave-uniform)
    const double fa = track[a];
    double fd = 0.0, fdd = 0.0;
    if (n >= 3) {
      if (a == 0) {
        fd = (-3.0 * track[0] + 4.0 * track[1] - track[2]) / (2.0 * T);
      } else if (a == n - 1) {
        fd = (3.0 * track[n - 1] - 4.0 * track[n - 2] + track[n - 3]) / (2.0 * T);
      } else {
        fd = (track[a + 1] - track[a - 1]) / (2.0 * T);
      }
      const int c = a == 0 ? 1 : (a == n - 1 ? n - 2 : a);
      fdd = (track[c + 1] - 2.0 * track[c] + track[c - 1]) / (T * T);
    } else if (n == 2) {
      fd = (track[1] - track[0]) / T;
    }
    const bool valid = __builtin_fabs(fdd) * T * T * T / 6.0 <= 1.0 && fa >= p.f_min && fd >= p.fdot_min;
    if (!valid) continue;
    const double x = fa * T;
    if (!(__builtin_fabs(x) < 1e9)) continue;          // far outside any row
    const double k0d = __builtin_rint(x);
    const int k0 = (int)k0d;
    if (k0 < 0 || k0 >= p.n_bins) continue;           // central bin outside the row: no contribution
    const float d0 = (float)(x - k0d);
    const float beta = (float)(fd * T * T);
    // template samples, Hann-windowed (lane holds m = lane + 64 q)
    float2 *s0 = buf[wave][0], *s1 = buf[wave][1];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = lane + 64 * q;
      const float u = (float)m * (1.0f / CH_M) - 0.5f;
      const float ph = beta * u * u + 2.0f * d0 * u;            // phase / pi
      float sn, cs;
      sincospif(ph, &sn, &cs);
      s0[m] = make_float2(win[m] * cs, win[m] * sn);
    }
    lds_wave_sync();
    const float2 *G = fft256(s0, s1, tw, lane);
    // window sums
    float nr = 0.0f, ni = 0.0f, dn = 0.0f;
    const size_t row = (size_t)a * p.pitch;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = lane + 64 * q;
      const int jo = jj - p.p_half;                                  // offset from k0
      const int k = k0 + jo;
      if (jj <= 2 * p.p_half && k >= 0 && k < p.n_bins) {
        const float2 h = G[jo & (CH_M - 1)];
        const float s = p.isq[k];
        const float2 z = p.Z[row + k];
        const float hr = h.x * s, hi = h.y * s;
        nr += z.x * hr + z.y * hi;                                   // conj(z) * h
        ni += z.x * hi - z.y * hr;
        dn += hr * hr + hi * hi;
      }
    }
    const double NR = wave_sum((double)nr), NI = wave_sum((double)ni), DN = wave_sum((double)dn);
    if (DN > 0.0) total += (NR * NR + NI * NI) / DN;
    lds_wave_sync();                   // the next segment's samples overwrite G
  }
  if (lane == 0) p.stat[j] = (float)total;
}

}  // namespace

hipError_t launch_chirp_prep(const double *psd, int n_bins, float *isq, TopkState *topk, hipStream_t stream) {
  const int blocks = (n_bins + CH_THREADS - 1) / CH_THREADS + (topk ? CH_RESET_PARTS : 0);
  hipLaunchKernelGGL(chirp_prep_kernel, dim3((unsigned)blocks), dim3(CH_THREADS), 0, stream, psd, n_bins, isq, topk);
  return hipGetLastError();
}

}  // namespace emri

using namespace emri;

namespace {

struct ChirpLayout {
  size_t isq, stat, topk, total;
};

ChirpLayout chirp_layout(int n_bins, int64_t n_tmpl, int top_k, bool stat_in_ws) {
  ChirpLayout L;
  size_t off = 0;
  L.isq = off;
  off += round_up((size_t)n_bins * sizeof(float), 256);
  L.stat = off;
  if (stat_in_ws) off += round_up((size_t)n_tmpl * sizeof(float), 256);
  L.topk = off;
  off += topk_workspace_bytes(top_k);
  L.total = off;
  return L;
}

int check_chirp(const emri_power *pw, int32_t K, int64_t n_tmpl, int32_t top_k, const chirp_opts *o) {
  if (!pw) return fail(EMRI_EINVAL, "sfts is NULL");
  if (pw->dtype != EMRI_C32) return fail(EMRI_EINVAL, "the linear-chirp statistic reads complex SFTs (EMRI_C32)");
  if (pw->n_seg < 0 || pw->n_bins < 1 || pw->row_pitch < pw->n_bins || (pw->row_pitch % 8) != 0)
    return fail(EMRI_EINVAL, "bad SFT geometry");
  if (!std::isfinite(pw->t_sft) || !(pw->t_sft > 0.0)) return fail(EMRI_EINVAL, "t_sft must be finite and > 0");
  if (pw->n_seg > CH_MAX_SEG) return fail(EMRI_EUNSUPPORTED, "at most %d segments", CH_MAX_SEG);
  if (K < 0 || K > EMRI_MAX_K) return fail(EMRI_EINVAL, "K = %d outside [0, %d]", K, EMRI_MAX_K);
  if (n_tmpl < 0 || n_tmpl > INT32_MAX) return fail(EMRI_EINVAL, "n_tmpl out of range");
  if (top_k < 0 || top_k > EMRI_MAX_TOPK) return fail(EMRI_EINVAL, "top_k out of range");
  if (o) {
    if (o->p_half < 0 || o->p_half > CH_MAX_P) return fail(EMRI_EUNSUPPORTED, "p_half must be in [0, %d]", CH_MAX_P);
    if (std::isnan(o->f_min) || std::isnan(o->fdot_min)) return fail(EMRI_EINVAL, "cut-offs must not be NaN");
    for (int i = 0; i < 4; ++i)
      if (o->reserved[i] != 0) return fail(EMRI_EINVAL, "chirp_opts.reserved must be zero");
  }
  return EMRI_OK;
}

}  // namespace

extern "C" int score_tracks_chirp_workspace_size(const emri_power *sfts, int32_t K, int64_t n_tmpl, int32_t top_k,
                                                 int32_t stat_in_workspace, size_t *bytes) {
  clear_error();
  if (!bytes) return fail(EMRI_EINVAL, "bytes is NULL");
  const int st = check_chirp(sfts, K, n_tmpl, top_k, nullptr);
  if (st) return st;
  *bytes = chirp_layout(sfts->n_bins, n_tmpl, top_k, stat_in_workspace != 0).total;
  return EMRI_OK;
}

extern "C" int score_tracks_chirp(const emri_power *sfts, const double *psd, const double *f0, const double *U,
                                  int32_t K, const float *coeffs, int64_t n_tmpl, int32_t top_k, float *stat,
                                  float *topk_val, int64_t *topk_idx, const chirp_opts *opts, void *workspace,
                                  size_t workspace_bytes, void *hip_stream) {
  clear_error();
  int st = check_chirp(sfts, K, n_tmpl, top_k, opts);
  if (st) return st;
  chirp_opts o{};
  o.p_half = CH_MAX_P;
  o.f_min = 3.1622776601683795e-4;       // 10^-3.5 Hz
  o.fdot_min = 1e-13;
  if (opts) o = *opts;
  if (!psd) return fail(EMRI_EINVAL, "psd is NULL");
  if (sfts->n_seg > 0 && (!sfts->data || !f0)) return fail(EMRI_EINVAL, "sfts->data or f0 is NULL");
  if (!U && K > 0 && sfts->n_seg > 0) return fail(EMRI_EINVAL, "U is NULL");
  if (!coeffs && K > 0 && n_tmpl > 0) return fail(EMRI_EINVAL, "coeffs is NULL");
  if (top_k > 0 && (!topk_val || !topk_idx)) return fail(EMRI_EINVAL, "topk_val/topk_idx are NULL");
  if (!workspace) return fail(EMRI_EINVAL, "workspace is NULL");
  const void *ptrs[] = {sfts->data, psd, f0, U, coeffs, stat, topk_val, topk_idx};
  for (const void *q : ptrs)
    if (q && !aligned16(q)) return fail(EMRI_EINVAL, "device pointers must be 16-byte aligned");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(EMRI_EINVAL, "workspace must be 256-byte aligned");
  const ChirpLayout L = chirp_layout(sfts->n_bins, n_tmpl, top_k, stat == nullptr);
  if (workspace_bytes < L.total)
    return fail(EMRI_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, L.total);
  int cus = 0;
  if ((st = device_cu_count(&cus)) != EMRI_OK) return st;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  char *ws = reinterpret_cast<char *>(workspace);
  float *isq = reinterpret_cast<float *>(ws + L.isq);
  float *stat_buf = stat ? stat : reinterpret_cast<float *>(ws + L.stat);
  hipError_t err = launch_chirp_prep(psd, sfts->n_bins, isq,
                                     top_k > 0 ? reinterpret_cast<TopkState *>(ws + L.topk) : nullptr, stream);
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "chirp prep launch: %s", hipGetErrorString(err));
  if (n_tmpl > 0) {
    ChirpParams p{};
    p.Z = reinterpret_cast<const float2 *>(sfts->data);
    p.isq = isq;
    p.f0 = f0;
    p.U = U;
    p.coeffs = coeffs;
    p.stat = stat_buf;
    p.n_tmpl = n_tmpl;
    p.t_sft = sfts->t_sft;
    p.f_min = o.f_min;
    p.fdot_min = o.fdot_min;
    p.pitch = sfts->row_pitch;
    p.n_seg = sfts->n_seg;
    p.n_bins = sfts->n_bins;
    p.K = K;
    p.p_half = o.p_half;
    const size_t lds = sizeof(double) * (size_t)CH_WAVES * (size_t)(sfts->n_seg > 0 ? sfts->n_seg : 1);
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(&chirp_score_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(chirp_score_kernel, dim3((unsigned)((n_tmpl + CH_WAVES - 1) / CH_WAVES)),
                         dim3(CH_THREADS), lds, stream, p);
      err = hipGetLastError();
    }
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "chirp launch: %s", hipGetErrorString(err));
  }
  if (top_k > 0) {
    err = launch_topk(stat_buf, n_tmpl, top_k, topk_val, topk_idx, ws + L.topk, cus, stream, 0);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "top-k launch: %s", hipGetErrorString(err));
  }
  return EMRI_OK;
}
