// Multi-harmonic form of the scoring kernel (Sec. IV proposes adding
// harmonics at a cost proportional to their number): harmonic h follows the
// searched track scaled by a fixed frequency ratio r_h, and every harmonic's
// nearest-bin power is summed over segments:
//     S[j] = sum_alpha sum_h P[alpha, rint(r_h x[j, alpha])],
//     x[j, alpha] = f0T[alpha] + sum_k c_jk UT[alpha, k]       (FP64)
// The layout and schedule are those of the plain kernel (persistent grid,
// lane-resident FP64 coefficients, spectrogram rows staged in LDS by the
// shared pipeline of staging.h): the K FMAs of a position are shared by the
// H harmonics, each harmonic adds one fused multiply-add that scales and
// rounds at once -- fma(x, r_h, 1.5*2^52 + B/E) rounds the exact product
// r_h x to an integer (half to even, B/E is even) and leaves B/E + rint(r_h x)
// in its low word -- one clamp onto the zero slots and one LDS gather from
// the row already staged for the searched harmonic.  Per segment the
// harmonics are added in order into the FP32 run (runs of 8 segments, FP64
// across runs).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <utility>

#include "common.h"
#include "score_internal.h"
#include "staging.h"

namespace emri {

namespace {

constexpr int HARM_MAX = 4;

struct HarmRatios {
  double r[HARM_MAX];
};

template <int K>
__device__ __forceinline__ void load_seg_h(const double *sp, double &f0t, double (&ut)[K]) {
  const_dptr sc = (const_dptr)sp;
  f0t = sc[0];
#pragma unroll
  for (int k = 0; k < K; ++k) ut[k] = sc[1 + k];
}

template <int K, int TPL, int H, bool WILD>
__device__ __forceinline__ void harmonic_addresses(const double (&c)[TPL][K], double f0t, const double (&ut)[K],
                                                   const BufConst &bc, const HarmRatios &hr, int (&addr)[TPL][H]) {
  double y[TPL];
#pragma unroll
  for (int s = 0; s < TPL; ++s) y[s] = f0t;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int s = 0; s < TPL; ++s) y[s] = __builtin_fma(c[s][k], ut[k], y[s]);
  }
#pragma unroll
  for (int s = 0; s < TPL; ++s) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
      double w;
      if constexpr (WILD) {
        const double t = y[s] * hr.r[h];
        w = (__builtin_fabs(t) < kWildLimit) ? __builtin_fma(y[s], hr.r[h], bc.magic) : bc.magic - 2.0;
      } else {
        w = __builtin_fma(y[s], hr.r[h], bc.magic);
      }
      addr[s][h] = clamp_i32(low_word(w), bc.lo, bc.hi);
    }
  }
}

template <int K, int TPL, int H, typename PT, bool WILD>
__device__ __forceinline__ void run_tile_h(const ScoreParams &p, const HarmRatios &hr, unsigned char *lds,
                                           const double (&c)[TPL][K], double (&sum)[TPL]) {
  constexpr int E = Elem<PT>::bytes;
  float acc[TPL];
#pragma unroll
  for (int s = 0; s < TPL; ++s) acc[s] = 0.0f;
  const Pipe pp = pipe_init<PT>(p);
  const int G = p.G;
  pipe_issue(p, pp, lds, 0, 0);
  pipe_publish<PT>(p, pp, lds, 0);
  int addr[TPL][H];
  double f0t, ut[K];
  if (p.n_seg > 0) {
    load_seg_h<K>(p.seg, f0t, ut);
    harmonic_addresses<K, TPL, H, WILD>(c, f0t, ut, buffer_consts<PT>(p, lds, 0, 0), hr, addr);
    load_seg_h<K>(p.seg + (p.n_seg > 1 ? p.seg_stride : 0), f0t, ut);
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);
  int half = 0;
  for (int r0 = 0; r0 < p.n_seg; r0 += G) {
    pipe_issue(p, pp, lds, r0 + G, half ^ 1);
    for (int i = 0; i < G; ++i) {
      const int r = r0 + i;
      if (r >= p.n_seg) break;
      typename Elem<PT>::raw_t v[TPL][H];
#pragma unroll
      for (int s = 0; s < TPL; ++s)
#pragma unroll
        for (int h = 0; h < H; ++h) v[s][h] = Elem<PT>::raw(E * addr[s][h]);
      // positions of segment r + 1 while these gathers are in flight, then the
      // constants of segment r + 2
      const int nh = i + 1 < G ? half : half ^ 1, nb = i + 1 < G ? i + 1 : 0;
      harmonic_addresses<K, TPL, H, WILD>(c, f0t, ut, buffer_consts<PT>(p, lds, nh, nb), hr, addr);
      __builtin_amdgcn_sched_barrier(0);
      load_seg_h<K>(p.seg + (size_t)(r + 2 < p.n_seg ? r + 2 : p.n_seg - 1) * p.seg_stride, f0t, ut);
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < TPL; ++s)
#pragma unroll
        for (int h = 0; h < H; ++h) acc[s] = Elem<PT>::add(acc[s], v[s][h], p.one);
      if ((r & 7) == 7 || r + 1 == p.n_seg) {
#pragma unroll
        for (int s = 0; s < TPL; ++s) {
          sum[s] += (double)acc[s];
          acc[s] = 0.0f;
        }
      }
    }
    pipe_publish<PT>(p, pp, lds, half ^ 1);
    half ^= 1;
  }
}

template <int K, int T, int H, typename PT>
__device__ __forceinline__ void score_tile_h(const ScoreParams &p, const HarmRatios &hr, double rmax,
                                             unsigned char *lds, int64_t t0, int64_t j_end, const double (&bound_u)[K],
                                             double bound_f0) {
  const int tid = threadIdx.x;
  double c[T][K];
  bool wild = false;
#pragma unroll
  for (int s = 0; s < T; ++s) {
    const int64_t j = t0 + (int64_t)s * SCORE_THREADS + tid;
    const bool live = j < j_end;
    double bnd = bound_f0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      c[s][k] = live ? (double)p.coeffs[(size_t)j * K + k] : 0.0;
      bnd += __builtin_fabs(c[s][k]) * bound_u[k];
    }
    wild |= !(bnd * rmax < 0.5 * kWildLimit);
  }
  double sum[T];
#pragma unroll
  for (int s = 0; s < T; ++s) sum[s] = 0.0;
  if (__any(wild))
    run_tile_h<K, T, H, PT, true>(p, hr, lds, c, sum);
  else
    run_tile_h<K, T, H, PT, false>(p, hr, lds, c, sum);
#pragma unroll
  for (int s = 0; s < T; ++s) {
    const int64_t j = t0 + (int64_t)s * SCORE_THREADS + tid;
    if (j < j_end) p.stat[j] = (float)sum[s];
  }
}

template <int K, int TPL, int H, typename PT>
__global__ __launch_bounds__(SCORE_THREADS) void score_harmonics_kernel(ScoreParams p, HarmRatios hr) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  init_lds(p, lds);
  const int64_t j_begin = (int64_t)blockIdx.x * p.per_block;
  const int64_t j_end = j_begin + p.per_block < p.n_tmpl ? j_begin + p.per_block : p.n_tmpl;
  const_dptr bnd_src = (const_dptr)p.bound;
  double bound_u[K];
#pragma unroll
  for (int k = 0; k < K; ++k) bound_u[k] = bnd_src[1 + k];
  const double bound_f0 = bnd_src[0];
  double rmax = 0.0;
#pragma unroll
  for (int h = 0; h < H; ++h) rmax = hr.r[h] > rmax ? hr.r[h] : rmax;
  constexpr int TAIL = (TPL + 1) / 2;
  for (int64_t t0 = j_begin; t0 < j_end; t0 += (int64_t)TPL * SCORE_THREADS) {
    if (TAIL < TPL && j_end - t0 <= (int64_t)TAIL * SCORE_THREADS) {
      score_tile_h<K, TAIL, H, PT>(p, hr, rmax, lds, t0, j_end, bound_u, bound_f0);
      break;
    }
    score_tile_h<K, TPL, H, PT>(p, hr, rmax, lds, t0, j_end, bound_u, bound_f0);
  }
}

// Templates per lane: the K coefficients (2K registers) plus, per harmonic,
// an address and a gathered value, within two waves' 256 registers per SIMD.
constexpr int tpl_h(int K, int H) {
  const int t = 176 / (2 * K + 2 * H + 3);
  return t > 12 ? 12 : (t < 1 ? 1 : t);
}

template <typename Kern>
hipError_t set_lds_h(Kern kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <int K, int H, typename PT>
hipError_t launch_h(const ScoreParams &p, const HarmRatios &hr, int grid, size_t lds, hipStream_t stream) {
  auto kern = score_harmonics_kernel<K, tpl_h(K, H), H, PT>;
  const hipError_t err = set_lds_h(kern, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(SCORE_THREADS), lds, stream, p, hr);
  return hipGetLastError();
}

template <int H, typename PT, int... Ks>
hipError_t dispatch_h(int K, const ScoreParams &p, const HarmRatios &hr, int grid, size_t lds, hipStream_t stream,
                      std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  (void)((K == Ks + 1 ? (err = launch_h<Ks + 1, H, PT>(p, hr, grid, lds, stream), true) : false) || ...);
  return err;
}

template <typename PT>
hipError_t dispatch_harm(int K, int H, const ScoreParams &p, const HarmRatios &hr, int grid, size_t lds,
                         hipStream_t stream) {
  using Ks = std::make_integer_sequence<int, HARMONICS_MAX_K>;
  switch (H) {
    case 1: return dispatch_h<1, PT>(K, p, hr, grid, lds, stream, Ks{});
    case 2: return dispatch_h<2, PT>(K, p, hr, grid, lds, stream, Ks{});
    case 3: return dispatch_h<3, PT>(K, p, hr, grid, lds, stream, Ks{});
    case 4: return dispatch_h<4, PT>(K, p, hr, grid, lds, stream, Ks{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_score_harmonics(const ScoreParams &p, int K, int dtype, int n_harm, const double *ratios, int grid,
                                  size_t lds, hipStream_t stream) {
  HarmRatios hr{};
  for (int h = 0; h < n_harm && h < HARM_MAX; ++h) hr.r[h] = ratios[h];
  if (dtype == EMRI_F32) return dispatch_harm<float>(K, n_harm, p, hr, grid, lds, stream);
  return dispatch_harm<__half>(K, n_harm, p, hr, grid, lds, stream);
}

}  // namespace emri
