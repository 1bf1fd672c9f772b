// The linear-chirp statistic (Sec. II B, Eqs. (4)-(7)): every segment's
// signal is a chirping sinusoid with the track's local frequency f and
// derivative fdot, its template SFT is evaluated over the 2P + 1 bins around
// rint(f T), and the phase- and amplitude-maximised inner product with the
// whitened data SFT is summed over the segments that pass the validity cut
// (|fddot| T^3 / 6 <= 1) and the cut-offs of Sec. II D.
//
// Per template (one wave):
//   * segments are taken 64 at a time, one per lane: the track values
//     f0 + sum_k c_k U[., k] (FP64) at the segment and its neighbours give f,
//     fdot and fddot (second-order finite differences: central inside,
//     one-sided at the ends for fdot, the neighbour's fddot at the ends), the
//     validity cut, k0 = rint(f T), d0 = f T - k0 and b = fdot T^2; the
//     segments that contribute are compacted by a ballot and taken one after
//     another, their parameters read from the owning lane;
//   * the template SFT of the unit chirp, Hann-windowed,
//         H_{k0 + j} ~ R(d0 - j, b),  R(d, b) = int cos^2(pi u) e^{2 pi i d u + i pi b u^2} du,
//     is the M = 256-point DFT of its samples
//     g_m = sin^2(pi m / M) e^{i pi (b u^2 + 2 d0 u)}, u = m / M - 1/2 (up to a
//     common factor; the integrand vanishes smoothly at both ends, so the
//     sum converges like the integral's aliased tail: relative error below
//     4e-7 for |b| <= 60 and P = 100), by a four-pass radix-4 Stockham FFT,
//     FP32: each lane holds the samples m = lane + 64 q (q = 0..3); their
//     phases form a quadratic sequence in q, so the lane evaluates the sample
//     at q = 0 and the step to q = 1 (two sine/cosine pairs) and takes the
//     rest by complex products, the step growing by the factor e^{i pi b / 8}
//     of the segment (evaluated once per segment in the parameter pass;
//     phase error a few units of 2^-24 of the phases, up to ~1e-5 rad);
//     these samples are the inputs
//     of its first butterfly, and keeps the outputs j = lane + 64 q of its
//     last; the two middle exchanges go through the wave's LDS buffer (padded
//     against bank conflicts), twiddles and window stay in registers;
//   * S_alpha = |sum_k conj(Z_k) H_k / sqrt(S_k)|^2 / sum_k |H_k|^2 / S_k over
//     the window's bins inside the row (FP32 products, FP32 tree sums across
//     the wave, the ratio in FP64), 0 when the central bin rint(f T) is
//     outside the row;
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
constexpr int CH_WAVES = 4;          // templates per workgroup
constexpr int CH_THREADS = 64 * CH_WAVES;
constexpr int CH_MAX_P = 100;        // 2P + 1 <= 201 bins
constexpr int CH_MAX_SEG = 2048;
static_assert(CH_M == 4 * 64, "four samples per lane");
static_assert(CH_MAX_P < CH_M / 2, "window within the FFT's unaliased bins");

// LDS slot of FFT element i: one float2 of padding after every four keeps
// each pass's writes and reads within two-way bank conflicts.
constexpr int lds_slot(int i) { return i + (i >> 2); }
// Raw buffer resources (stride 0): word 3 as the gfx9 family takes it; a
// load at or past num_records bytes returns zero.
constexpr int CH_RSRC_WORD3 = 0x00020000;
constexpr unsigned CH_OUTSIDE = 0x80000000u;
constexpr int CH_MAX_BINS = 1 << 27;   // byte offsets of bins and of CH_OUTSIDE + 8 k0 stay below 2^32
constexpr int CH_LDS = lds_slot(CH_M - 1) + 1;

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

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// y_r = sum_q v_q e^{-2 pi i q r / 4}
__device__ __forceinline__ void butterfly4(float2 v[4]) {
  const float2 s02 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
  const float2 d02 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
  const float2 s13 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
  const float2 d13 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
  v[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
  v[1] = make_float2(d02.x + d13.y, d02.y - d13.x);          // d02 - i d13
  v[2] = make_float2(s02.x - s13.x, s02.y - s13.y);
  v[3] = make_float2(d02.x - d13.y, d02.y + d13.x);          // d02 + i d13
}

__device__ __forceinline__ void lds_wave_sync() {
  // the wave's LDS writes are complete before any lane reads another lane's data
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}

// Sum over the wave, FP32, as a tree: quad swaps, the half-row and row
// mirrors (every lane then holds its row of 16), then rows 0 + 1 and 2 + 3
// by the row-15 broadcast and all four by the row-31 broadcast, which lands
// in the last row; the result is read from lane 63.
__device__ __forceinline__ float wave_total(float v) {
  v += dpp<0xB1>(v);                   // quad_perm [1, 0, 3, 2]
  v += dpp<0x4E>(v);                   // quad_perm [2, 3, 0, 1]
  v += dpp<0x141>(v);                  // row_half_mirror
  v += dpp<0x140>(v);                  // row_mirror
  v += dpp<0x142, 0xA>(v);             // row_bcast15 into rows 1 and 3 (rows 0 and 2 add zero)
  v += dpp<0x143, 0xC>(v);             // row_bcast31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// sin(pi x) and cos(pi x) for finite x of moderate size (|2x| < 2^31): x is
// reduced to r = x - n/2, |r| <= 1/4, exactly; t = pi r; Taylor polynomials
// of degree 9 (sine) and 8 (cosine) in t leave a truncation below 2e-9 on
// |t| <= pi/4; the quadrant n mod 4 swaps and negates.  Absolute error about
// 1.3 units of 2^-24 in FP32.
__device__ __forceinline__ void sincospi_reduced(float x, float *sn, float *cs) {
  const float n = __builtin_rintf(2.0f * x);
  const float t = fmaf(n, -0.5f, x) * 3.14159265358979f;
  const float z = t * t;
  float ps = fmaf(z, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(z, ps, 1.0f / 120.0f);
  ps = fmaf(z, ps, -1.0f / 6.0f);
  const float s = fmaf(t * z, ps, t);
  float pc = fmaf(z, 1.0f / 40320.0f, -1.0f / 720.0f);
  pc = fmaf(z, pc, 1.0f / 24.0f);
  pc = fmaf(z, pc, -0.5f);
  const float c = fmaf(z, pc, 1.0f);
  const int q = (int)n;
  const bool swap = (q & 1) != 0;
  const float a = swap ? c : s, b = swap ? s : c;
  *sn = __int_as_float(__float_as_int(a) ^ ((q & 2) << 30));
  *cs = __int_as_float(__float_as_int(b) ^ (((q + 1) & 2) << 30));
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
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
  __shared__ float2 lds[CH_WAVES][CH_LDS];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  const int64_t j = (int64_t)blockIdx.x * CH_WAVES + wave;
  if (j >= p.n_tmpl) return;           // no block-wide barrier in this kernel
  float2 *buf = lds[wave];

  // lane constants: window and sample offsets, twiddles of passes 1..3,
  // LDS slots of each pass, window offsets j of the lane's outputs
  float win[4], uq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = lane + 64 * q;
    const double w = sinpi((double)m / CH_M);
    win[q] = (float)(w * w);
    uq[q] = (float)m * (1.0f / CH_M) - 0.5f;
  }
  float2 tw[3][3];
#pragma unroll
  for (int ps = 1; ps < 4; ++ps) {
    const int ns = 1 << (2 * ps);
    const int k = lane & (ns - 1);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      double sn, cs;
      sincospi(-2.0 * (double)(r * k) / (double)(4 * ns), &sn, &cs);
      tw[ps - 1][r - 1] = make_float2((float)cs, (float)sn);
    }
  }
  const int rd = lds_slot(lane);                                        // + 80 r: element lane + 64 r
  const int wr0 = lds_slot(4 * lane);                                   // + r: element 4 lane + r
  const int wr1 = lds_slot(16 * (lane >> 2) + (lane & 3));              // + 5 r: element ... + 4 r
  const int wr2 = lds_slot(64 * (lane >> 4) + (lane & 15));             // + 20 r: element ... + 16 r
  // byte offsets, from the central bin, of the bins of the lane's outputs
  // (output lane + 64 r is bin offset jo); outside the window they carry
  // 2^31, which keeps every such load past the end of its buffer
  unsigned zoff[4], ioff[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jo = lane + 64 * r - (r >= 2 ? CH_M : 0);
    const bool in_win = jo >= -p.p_half && jo <= p.p_half;
    zoff[r] = in_win ? (unsigned)jo * 8u : CH_OUTSIDE;
    ioff[r] = in_win ? (unsigned)jo * 4u : CH_OUTSIDE;
  }
  // bins outside the row read as zero: raw buffer loads past num_records
  const __amdgpu_buffer_rsrc_t isq_rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void *)p.isq, (short)0, p.n_bins * 4, CH_RSRC_WORD3);

  const double T = p.t_sft;
  const int n = p.n_seg, K = p.K;
  const float *cj = p.coeffs + (size_t)j * K;
  double num = 0.0, den = 0.0;          // this lane's slot: one segment of the chunk
  double total = 0.0;                   // this lane's share of S
  for (int base = 0; base < n; base += 64) {
    // ---- this chunk's segment parameters, one segment per lane ----
    const int a = base + lane;
    bool use = false;
    int k0v = 0;
    float d0v = 0.0f, bv = 0.0f, qsv = 0.0f, qcv = 1.0f;
    if (a < n) {
      auto track = [&](int i) {
        double f = p.f0[i];
        for (int k = 0; k < K; ++k) f = __builtin_fma((double)cj[k], p.U[(size_t)i * K + k], f);
        return f;
      };
      double fa, fd = 0.0, fdd = 0.0;
      if (n >= 3) {
        const int c = a < 1 ? 1 : (a > n - 2 ? n - 2 : a);
        const double fm = track(c - 1), fc = track(c), fp = track(c + 1);
        if (a == 0) {
          fa = fm;
          fd = (-3.0 * fm + 4.0 * fc - fp) / (2.0 * T);
        } else if (a == n - 1) {
          fa = fp;
          fd = (3.0 * fp - 4.0 * fc + fm) / (2.0 * T);
        } else {
          fa = fc;
          fd = (fp - fm) / (2.0 * T);
        }
        fdd = (fp - 2.0 * fc + fm) / (T * T);
      } else if (n == 2) {
        const double g0 = track(0), g1 = track(1);
        fa = a == 0 ? g0 : g1;
        fd = (g1 - g0) / T;
      } else {
        fa = track(0);
      }
      const bool valid = __builtin_fabs(fdd) * T * T * T / 6.0 <= 1.0 && fa >= p.f_min && fd >= p.fdot_min;
      const double x = fa * T;
      if (valid && __builtin_fabs(x) < 1e9) {                           // else far outside any row
        const double k0d = __builtin_rint(x);
        k0v = (int)k0d;
        d0v = (float)(x - k0d);
        bv = (float)(fd * T * T);
        // central bin outside the row, or b beyond FP32: no contribution
        use = k0v >= 0 && k0v < p.n_bins && __builtin_fabsf(bv) <= 3.4028234663852886e38f;
        if (use) sincospi_reduced(bv * 0.125f, &qsv, &qcv);                 // e^{i pi b / 8}: second difference of the phase
      }
    }
    uint64_t todo = __ballot(use);
    // ---- the chunk's contributing segments, one after another ----
    while (todo) {
      const int l = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int k0 = __builtin_amdgcn_readlane(k0v, l);
      const float d0 = readlane_f(d0v, l), beta = readlane_f(bv, l);
      const float2 Qs = make_float2(readlane_f(qcv, l), readlane_f(qsv, l));
      const __amdgpu_buffer_rsrc_t zrow = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(p.Z + (size_t)(base + l) * p.pitch), (short)0, p.n_bins * 8, CH_RSRC_WORD3);
      // the window's data and weights depend on k0 only: their loads go out
      // first and land while the samples and the FFT are computed
      float sw[4];
      float2 zw[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sw[r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(isq_rsrc, (unsigned)k0 * 4u + ioff[r], 0, 0));
        const auto zb = __builtin_amdgcn_raw_buffer_load_b64(zrow, (unsigned)k0 * 8u + zoff[r], 0, 0);
        zw[r] = make_float2(__uint_as_float(zb[0]), __uint_as_float(zb[1]));
      }
      __builtin_amdgcn_sched_barrier(0);
      // samples (lane holds m = lane + 64 q) and the first butterfly
      float2 v[4];
      {
        // phase / pi at u0 and its first difference to u0 + 1/4; later
        // differences grow by b / 8, so the samples follow by products
        const float u0 = uq[0];
        const float ph = u0 * fmaf(beta, u0, 2.0f * d0);
        const float dph = fmaf(beta, 2.0f * u0 + 0.25f, 2.0f * d0) * 0.25f;
        float sn, cs, rs, rc;
        sincospi_reduced(ph, &sn, &cs);
        sincospi_reduced(dph, &rs, &rc);
        float2 e = make_float2(cs, sn), r = make_float2(rc, rs);
        v[0] = make_float2(win[0] * e.x, win[0] * e.y);
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          e = cmul(e, r);
          if (q < 3) r = cmul(r, Qs);
          v[q] = make_float2(win[q] * e.x, win[q] * e.y);
        }
      }
      butterfly4(v);
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[wr0 + r] = v[r];
      lds_wave_sync();
      // pass 1 (stride 4) and pass 2 (stride 16), in place
#pragma unroll
      for (int ps = 1; ps < 3; ++ps) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = buf[rd + 80 * r];
#pragma unroll
        for (int r = 1; r < 4; ++r) v[r] = cmul(v[r], tw[ps - 1][r - 1]);
        butterfly4(v);
        if (ps == 1) {
#pragma unroll
          for (int r = 0; r < 4; ++r) buf[wr1 + 5 * r] = v[r];
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) buf[wr2 + 20 * r] = v[r];
        }
        lds_wave_sync();
      }
      // pass 3 (stride 64): outputs j = lane + 64 r stay in the lane
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = buf[rd + 80 * r];
#pragma unroll
      for (int r = 1; r < 4; ++r) v[r] = cmul(v[r], tw[2][r - 1]);
      butterfly4(v);
      // window sums over the lane's bins (outside the window or the row: zero)
      float nr = 0.0f, ni = 0.0f, dn = 0.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float s = sw[r];
        const float zx = zw[r].x, zy = zw[r].y;
        const float hr = v[r].x * s, hi = v[r].y * s;
        nr = fmaf(zx, hr, fmaf(zy, hi, nr));                            // conj(z) * h
        ni = fmaf(zx, hi, fmaf(-zy, hr, ni));
        dn = fmaf(hr, hr, fmaf(hi, hi, dn));
      }
      const double NR = wave_total(nr), NI = wave_total(ni), DN = wave_total(dn);   // FP32 sums
      if (lane == l) {
        num = NR * NR + NI * NI;
        den = DN;
      }
      asm volatile("" ::: "memory");   // the next segment's first writes follow this segment's last reads
    }
    if (use && den > 0.0) total += num / den;
    num = 0.0;
    den = 0.0;
  }
  // S over the lanes' shares, FP64
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
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
  if (pw->n_bins > CH_MAX_BINS) return fail(EMRI_EUNSUPPORTED, "at most %d bins", CH_MAX_BINS);
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
    hipLaunchKernelGGL(chirp_score_kernel, dim3((unsigned)((n_tmpl + CH_WAVES - 1) / CH_WAVES)), dim3(CH_THREADS), 0,
                       stream, p);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "chirp launch: %s", hipGetErrorString(err));
  }
  if (top_k > 0) {
    err = launch_topk(stat_buf, n_tmpl, top_k, topk_val, topk_idx, ws + L.topk, cus, stream, 0);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "top-k launch: %s", hipGetErrorString(err));
  }
  return EMRI_OK;
}
