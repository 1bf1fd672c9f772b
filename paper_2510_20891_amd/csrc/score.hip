// score_tracks kernels: track reconstruction, nearest-bin power gather and
// segment reduction in one pass (Eq. (6) in its nearest-bin limit, tracks from
// the basis product of Eq. (10), bin width 1/T_SFT of Sec. II B).
//
// Layout and schedule (MI355X / gfx950):
//   * A persistent grid of one workgroup per CU (NT = 1024 threads for a
//     standalone launch, 512 in the batched one).  Workgroup g owns a
//     contiguous range of templates and walks it in tiles of TPL*NT templates:
//     lane l holds TPL templates (j = tile + s*NT + l), their K coefficients
//     widened to FP64 and kept in VGPRs for the whole tile.
//   * Each power row P[alpha, 0..n_bins) is staged in LDS by asynchronous
//     global->LDS copies (global_load_lds_dwordx4, 1 KB per wave instruction).
//     Two halves of G = 1, 2 or 4 row buffers alternate: while the G rows of one
//     step are gathered from, the next G rows are copied into the other half.  Every workgroup walks the rows in the same
//     order, so the 32 CUs of an XCD share each row in their L2.
//   * Per (template, segment), with E = element size in bytes and B = the LDS
//     byte address of bin 0 of the current buffer:
//       x    = f0T[alpha] + sum_k c_k UT[alpha,k]        FP64 fused multiply-adds
//       w    = low word of (x + 1.5*2^52 + B/E)         = B/E + rint(x)
//       w    = med3(w, B/E + k_min - 1, B/E + k_max + 1)
//       acc += P at LDS byte address E*w
//     Adding the constant makes the FPU round x to an integer (half to even,
//     since B/E is even) and leaves that integer, offset by B/E, in the low
//     word: the FPU's own rounding places the bin.  Bins outside [k_min, k_max]
//     clamp onto the two slots next to the range, which hold zeros.  f0T = f0*T
//     and UT = U*T are wave-uniform and come from scalar loads.
//   * The statistic is summed in FP32 over runs of 8 segments and in FP64
//     across runs; the fixed order makes results independent of the launch.
//   * Templates whose |x| could reach 2^26 (huge or non-finite coefficients,
//     non-finite f0/U) are detected per wave from a cheap bound and take a path
//     that maps such positions (never inside a spectrogram row) to bin -2
//     before rounding, so they contribute nothing.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "common.h"
#include "score_internal.h"
#include "topk_internal.h"
#include "topk_device.h"
#include "staging.h"

namespace emri {

namespace {

template <int K>
__device__ __forceinline__ void load_segment(const double *sp, double &f0t, double (&ut)[K > 0 ? K : 1]) {
  const_dptr sc = (const_dptr)sp;
  f0t = sc[0];
#pragma unroll
  for (int k = 0; k < K; ++k) ut[k] = sc[1 + k];
}

// LDS element addresses of the TPL templates' bins in one segment.  k-outer
// order keeps TPL independent FMA chains in flight (FP64 FMA latency is longer
// than its issue time).
template <int K, int TPL, bool WILD>
__device__ __forceinline__ void bin_addresses(const double (&c)[TPL][K > 0 ? K : 1], double f0t,
                                              const double (&ut)[K > 0 ? K : 1], const BufConst &bc,
                                              int (&addr)[TPL]) {
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
    double ys = y[s];
    if constexpr (WILD) ys = (__builtin_fabs(ys) < kWildLimit) ? ys : -2.0;
    addr[s] = clamp_i32(low_word(ys + bc.magic), bc.lo, bc.hi);
  }
}

// One tile of TPL slots of 512 templates against every segment.  Software
// pipelined per wave: the gathers of segment r are in flight while the bins of
// segment r+1 are computed (its constants were loaded one segment earlier).
template <int K, int TPL, typename PT, bool WILD>
__device__ __forceinline__ void run_tile(const ScoreParams &p, unsigned char *lds,
                                         const double (&c)[TPL][K > 0 ? K : 1], double (&sum)[TPL]) {
  constexpr int E = Elem<PT>::bytes;
  float acc[TPL];
#pragma unroll
  for (int s = 0; s < TPL; ++s) acc[s] = 0.0f;
  const Pipe pp = pipe_init<PT>(p);
  const int G = p.G;
  if (pp.wave < SCORE_WAVES) pipe_issue(p, pp, lds, 0, 0);
  pipe_publish<PT>(p, pp, lds, 0);
  int addr[TPL];
  double f0t, ut[K > 0 ? K : 1];
  if (p.n_seg > 0) {
    load_segment<K>(p.seg, f0t, ut);
    bin_addresses<K, TPL, WILD>(c, f0t, ut, buffer_consts<PT>(p, lds, 0, 0), addr);
    load_segment<K>(p.seg + (p.n_seg > 1 ? p.seg_stride : 0), f0t, ut);
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);     // lgkmcnt(0): nothing scalar in flight entering the loop
  int half = 0;
  for (int r0 = 0; r0 < p.n_seg; r0 += G) {
    if (pp.wave < SCORE_WAVES) pipe_issue(p, pp, lds, r0 + G, half ^ 1);
    for (int i = 0; i < G; ++i) {
      const int r = r0 + i;
      if (r >= p.n_seg) break;
      typename Elem<PT>::raw_t v[TPL];
#pragma unroll
      for (int s = 0; s < TPL; ++s) v[s] = Elem<PT>::raw(E * addr[s]);
      // The bins of segment r+1 (for the last segment these are clamped, unused
      // addresses) and the constants of segment r+2.  Up to K = 8 the constants
      // go to a second set of scalar registers before the FMAs, so that their
      // loads are in flight meanwhile; above, two sets would crowd the scalar
      // registers (measured: K = 8 3-5 % faster, K = 16 17 % slower), and they
      // are loaded after the FMAs into the set just used.
      const int nh = i + 1 < G ? half : half ^ 1, nb = i + 1 < G ? i + 1 : 0;
      const double *next = p.seg + (size_t)(r + 2 < p.n_seg ? r + 2 : p.n_seg - 1) * p.seg_stride;
      if constexpr (K <= 8) {
        double f0n, un[K > 0 ? K : 1];
        load_segment<K>(next, f0n, un);
        __builtin_amdgcn_sched_barrier(0);
        bin_addresses<K, TPL, WILD>(c, f0t, ut, buffer_consts<PT>(p, lds, nh, nb), addr);
        __builtin_amdgcn_sched_barrier(0);
        f0t = f0n;
#pragma unroll
        for (int k = 0; k < (K > 0 ? K : 1); ++k) ut[k] = un[k];
      } else {
        bin_addresses<K, TPL, WILD>(c, f0t, ut, buffer_consts<PT>(p, lds, nh, nb), addr);
        __builtin_amdgcn_sched_barrier(0);
        load_segment<K>(next, f0t, ut);
      }
      // lgkmcnt(0): this segment's gathers and the scalar loads; the next
      // segment's FMAs then start without waiting for its own gathers.
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < TPL; ++s) acc[s] = Elem<PT>::add(acc[s], v[s], p.one);
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

// One tile of T slots (T x NT templates starting at t0, clipped to j_end; NT
// threads per workgroup).
template <int K, int T, typename PT, int NT = SCORE_THREADS>
__device__ __forceinline__ void score_tile(const ScoreParams &p, unsigned char *lds, int64_t t0, int64_t j_end,
                                           const double (&bound_u)[K > 0 ? K : 1], double bound_f0) {
  const int tid = threadIdx.x;
  double c[T][K > 0 ? K : 1];
  bool wild = false;
#pragma unroll
  for (int s = 0; s < T; ++s) {
    const int64_t j = t0 + (int64_t)s * NT + tid;
    const bool live = j < j_end;
    float cf[K > 0 ? K : 1];
    if constexpr (K % 4 == 0) {
#pragma unroll
      for (int k = 0; k < K; k += 4) {
        const float4 v = live ? reinterpret_cast<const float4 *>(p.coeffs + (size_t)j * K)[k / 4]
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        cf[k] = v.x; cf[k + 1] = v.y; cf[k + 2] = v.z; cf[k + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) cf[k] = live ? p.coeffs[(size_t)j * K + k] : 0.0f;
    }
    double bnd = bound_f0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      c[s][k] = (double)cf[k];
      bnd += __builtin_fabs(c[s][k]) * bound_u[k];
    }
    wild |= !(bnd < 0.5 * kWildLimit);
  }
  double sum[T];
#pragma unroll
  for (int s = 0; s < T; ++s) sum[s] = 0.0;
  if (__any(wild))
    run_tile<K, T, PT, true>(p, lds, c, sum);
  else
    run_tile<K, T, PT, false>(p, lds, c, sum);
#pragma unroll
  for (int s = 0; s < T; ++s) {
    const int64_t j = t0 + (int64_t)s * NT + tid;
    if (j < j_end) p.stat[j] = (float)sum[s];
  }
}

// Score templates [j_begin, j_end) of one stream (the workgroup's share) in
// tiles of TPL slots; a last tile that fits in half as many slots runs with
// half (the per-template arithmetic and order do not depend on the tile).
template <int K, int TPL, typename PT, int NT = SCORE_THREADS>
__device__ __forceinline__ void score_range(const ScoreParams &p, unsigned char *lds, int64_t j_begin,
                                            int64_t j_end) {
  constexpr int TAIL = (TPL + 1) / 2;
  const_dptr bnd_src = (const_dptr)p.bound;
  double bound_u[K > 0 ? K : 1];
#pragma unroll
  for (int k = 0; k < K; ++k) bound_u[k] = bnd_src[1 + k];
  const double bound_f0 = bnd_src[0];
  for (int64_t t0 = j_begin; t0 < j_end; t0 += (int64_t)TPL * NT) {
    if (TAIL < TPL && j_end - t0 <= (int64_t)TAIL * NT) {
      score_tile<K, TAIL, PT, NT>(p, lds, t0, j_end, bound_u, bound_f0);
      break;
    }
    score_tile<K, TPL, PT, NT>(p, lds, t0, j_end, bound_u, bound_f0);
  }
}

// The first top-k key pass over this workgroup's own statistics (standalone
// plain launches with a top-k; the top-k launch then starts at its second
// pass).  The staging rows are no longer needed, so the LDS holds the
// histogram of the 12-bit leading key digit, counted as the top-k's own first
// pass does (an 8-bin register window per wave); the workgroups merge it in
// two levels and the last one picks the digit.
template <int NT>
__device__ void first_key_pass_of_range(const ScoreParams &p, unsigned char *lds, int64_t j_begin, int64_t j_end) {
  constexpr int SHIFT = 20, WIDTH = 12;
  constexpr uint32_t MASK = (1u << WIDTH) - 1u;
  uint32_t *lh = reinterpret_cast<uint32_t *>(lds);
  __syncthreads();               // every statistic of this workgroup written, every row read
  clear_hist(lh, TOPK_HIST);
  const int lane = (int)(threadIdx.x & 63);
  uint32_t base = 0u;
  uint64_t packed = 0ull;
  int count = 0;
  bool have_base = false;
  // wave-uniform trip count: lanes past the end count nothing; eight loads
  // in flight per lane (the loop is otherwise latency-bound)
  constexpr int U = 8;
  const int64_t step = (int64_t)blockDim.x;
  for (int64_t j0 = j_begin + (int64_t)(threadIdx.x & ~63u); j0 < j_end; j0 += U * step) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * step + lane;
      v[u] = j < j_end ? p.stat[j] : 0.0f;
    }
    if (!have_base) {            // the wave's first lane is live here
      const uint32_t b0 = __builtin_amdgcn_readfirstlane((order_key(v[0]) >> SHIFT) & MASK);
      base = b0 >= 3u ? b0 - 3u : 0u;
      have_base = true;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = j0 + u * step + lane < j_end;
      const uint32_t bin = (order_key(v[u]) >> SHIFT) & MASK;
      const uint32_t d = bin - base;
      packed += (live && d < 8u) ? 1ull << (8u * d) : 0ull;
      if (live && d >= 8u) atomicAdd(&lh[bin], 1u);
    }
    count += U;
    if (count > 255 - U) {       // 8-bit fields
      add_window(lh, base, packed);
      packed = 0ull;
      count = 0;
    }
  }
  if (count > 0) add_window(lh, base, packed);
  flush_hist(lh, p.topk->ghist[blockIdx.x % TOPK_GROUPS], TOPK_HIST);
  if (finish_pass<NT>(p.topk, TOPK_HIST, (int)blockIdx.x, (int)gridDim.x)) {
    TopkJob job{};
    job.st = p.topk;
    job.kk = p.topk_kk;
    select_digit<true, NT>(job, lh, SHIFT, WIDTH, true, false, false);
  }
}

// The standalone kernel runs FAST_THREADS-thread workgroups (four waves per
// SIMD with 128 VGPRs each, half the templates per lane of the 512-thread
// batched kernel, so a tile is as large): twice the waves to hide the FP64
// multiply-add chains and the gathers behind.  The first SCORE_WAVES waves
// stage the rows.  One-year, K = 8: 1e7 templates FP32 1.49 -> 1.39 ms, 1e8
// templates 12.85 -> 11.28 ms; K = 16, 1e8: 26.8 -> 23.2 ms (FP32).
constexpr int FAST_THREADS = 1024;

template <int K, int TPL, typename PT>
__global__ __launch_bounds__(FAST_THREADS) void score_fast_kernel(ScoreParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  init_lds(p, lds);
  const int64_t j_begin = (int64_t)blockIdx.x * p.per_block;
  const int64_t j_end = j_begin + p.per_block < p.n_tmpl ? j_begin + p.per_block : p.n_tmpl;
  score_range<K, TPL, PT, FAST_THREADS>(p, lds, j_begin, j_end);
  if (p.topk) first_key_pass_of_range<FAST_THREADS>(p, lds, j_begin, j_end);
}

// Batched form: one persistent launch over many streams.  Workgroups claim
// work items (a range of one stream's templates) until the table is
// exhausted; every stream carries its own spectrogram, constants, bin range
// and staging geometry.
template <int K, int TPL, typename PT>
__global__ __launch_bounds__(SCORE_THREADS) void score_batched_kernel(const ScoreParams *__restrict__ params,
                                                                      const BatchItem *__restrict__ items,
                                                                      int n_items, int *counter) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ int slot;
  for (;;) {
    const int it = claim_item(counter, &slot);
    if (it >= n_items) break;
    const BatchItem item = load_uniform(items + it);
    const ScoreParams p = load_uniform(params + item.stream);
    init_lds(p, lds);
    score_range<K, TPL, PT>(p, lds, item.begin, item.end);
  }
}

// Validation variant: one template per lane and runtime K; it also records the
// chosen bins and counts near-ties.  Same arithmetic and summation order as the
// fast kernel, so the statistics agree bit for bit.
template <typename PT>
__global__ __launch_bounds__(SCORE_THREADS) void score_validate_kernel(ScoreParams p, int K) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  constexpr int E = Elem<PT>::bytes;
  const int tid = threadIdx.x;
  init_lds(p, lds);
  const int64_t j_begin = (int64_t)blockIdx.x * p.per_block;
  const int64_t j_end = j_begin + p.per_block < p.n_tmpl ? j_begin + p.per_block : p.n_tmpl;
  unsigned long long near = 0;
  for (int64_t t0 = j_begin; t0 < j_end; t0 += SCORE_THREADS) {
    const int64_t j = t0 + tid;
    const bool live = j < j_end;
    double c[EMRI_MAX_K];
#pragma unroll
    for (int k = 0; k < EMRI_MAX_K; ++k) c[k] = (k < K && live) ? (double)p.coeffs[(size_t)j * K + k] : 0.0;
    double sum = 0.0;
    float acc = 0.0f;
    const Pipe pp = pipe_init<PT>(p);
    pipe_issue(p, pp, lds, 0, 0);
    pipe_publish<PT>(p, pp, lds, 0);
    int half = 0;
    for (int r0 = 0; r0 < p.n_seg; r0 += p.G) {
      pipe_issue(p, pp, lds, r0 + p.G, half ^ 1);
      for (int i = 0; i < p.G && r0 + i < p.n_seg; ++i) {
        const int a = r0 + i;
        const_dptr sc = (const_dptr)(p.seg + (size_t)a * p.seg_stride);
        double y = sc[0];
#pragma unroll
        for (int k = 0; k < EMRI_MAX_K; ++k)
          if (k < K) y = __builtin_fma(c[k], sc[1 + k], y);
        if (__builtin_fabs(y) <= 1.7976931348623157e308 && live) {
          const double fr = y - __builtin_floor(y);
          if (__builtin_fabs(fr - 0.5) < kNearTie) ++near;
        }
        const double ys = (__builtin_fabs(y) < kWildLimit) ? y : -2.0;
        const BufConst bc = buffer_consts<PT>(p, lds, half, i);
        const int word = low_word(ys + bc.magic);
        const int b = word - bc.base;
        acc = Elem<PT>::add(acc, Elem<PT>::raw(E * clamp_i32(word, bc.lo, bc.hi)), p.one);
        if (live && p.bins) p.bins[(size_t)j * p.n_seg + a] = (b >= p.k_min && b <= p.k_max) ? b : -1;
        if ((a & 7) == 7 || a + 1 == p.n_seg) {
          sum += (double)acc;
          acc = 0.0f;
        }
      }
      pipe_publish<PT>(p, pp, lds, half ^ 1);
      half ^= 1;
    }
    if (live && p.stat) p.stat[j] = (float)sum;
  }
  if (p.near_tie && near) atomicAdd(p.near_tie, near);
}

// Per-segment constants f0*T, U*T (FP64) and the bounds of the wild-template
// test: bound[0] = max |f0 T|, bound[1+k] = max_alpha |U[alpha,k] T| (+inf if
// an entry is not finite).  Also clears the near-tie counter and, with
// reset_topk, the top-k state of the call.  One workgroup of 256 threads.
__device__ __forceinline__ double abs_bound(double v) {
  const double av = __builtin_fabs(v);
  return av <= 1.7976931348623157e308 ? av : __builtin_inf();     // NaN and inf: +inf
}

__device__ __forceinline__ void prep_one(const PrepJob &job, bool reset_topk) {
  __shared__ double red[4][EMRI_MAX_K + 1];
  const double *f0 = job.f0, *U = job.U;
  const int K = job.K, n_seg = job.n_seg, stride = job.seg_stride;
  const double t_sft = job.t_sft;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0 && job.near_tie) *job.near_tie = 0ull;
  if (threadIdx.x == 0 && job.redo) *job.redo = 0u;
  if (job.topk && reset_topk) topk_state_reset(job.topk, 0, 1);
  for (int a = threadIdx.x; a < n_seg; a += blockDim.x) {
    job.seg[(size_t)a * stride] = f0[a] * t_sft;
    for (int k = 0; k < K; ++k) job.seg[(size_t)a * stride + 1 + k] = U[(size_t)a * K + k] * t_sft;
  }
  // column maxima eight columns at a time, so that the eight shuffle chains
  // of a group run interleaved
  for (int c0 = 0; c0 <= K; c0 += 8) {
    double m[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) m[j] = 0.0;
    for (int a = threadIdx.x; a < n_seg; a += blockDim.x) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int col = c0 + j;
        if (col <= K) {
          const double b = abs_bound(col == 0 ? f0[a] * t_sft : U[(size_t)a * K + col - 1] * t_sft);
          m[j] = b > m[j] ? b : m[j];
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double o = __shfl_xor(m[j], off, 64);
        m[j] = o > m[j] ? o : m[j];
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (c0 + j <= K) red[wave][c0 + j] = m[j];
    }
  }
  __syncthreads();
  if (threadIdx.x <= K) {
    double m = red[0][threadIdx.x];
    for (int w = 1; w < 4; ++w) m = red[w][threadIdx.x] > m ? red[w][threadIdx.x] : m;
    job.bound[threadIdx.x] = m;
  }
  if (job.mtab) {
    // mixed-precision tables: U*T as three BF16 pieces (u0 + u1 + u2 carries
    // about 24 bits; each piece is the rounded FP64 remainder of the previous
    // ones), and f0*T split into an even integer and a fraction
    const int KG = mixed_groups(K), n4 = (n_seg + 3) & ~3;
    unsigned short *tab = reinterpret_cast<unsigned short *>(job.mtab);
    for (int e = threadIdx.x; e < n4 * 4 * KG; e += blockDim.x) {
      const int a = e / (4 * KG), k = e % (4 * KG);
      const double x = (a < n_seg && k < K) ? U[(size_t)a * K + k] * t_sft : 0.0;
      const unsigned short p0 = bf16_rne((float)x);
      const double r1 = x - (double)bf16_value(p0);
      const unsigned short p1 = bf16_rne((float)r1);
      const double r2 = r1 - (double)bf16_value(p1);
      const unsigned short p2 = bf16_rne((float)r2);
      unsigned short *row = tab + (size_t)a * (3 * KG * 4) + (k >> 2) * 4 + (k & 3);
      row[0] = p0;
      row[KG * 4] = p1;
      row[2 * KG * 4] = p2;
    }
    MixedSeg *ms = reinterpret_cast<MixedSeg *>(job.mseg);
    for (int a = threadIdx.x; a < n4; a += blockDim.x) {
      MixedSeg m;
      m.I = 0.0;
      m.phi = 0.0f;
      m.M = 12582912.0f;
      if (a < n_seg) {
        const double v = f0[a] * t_sft;
        m.I = 2.0 * __builtin_rint(0.5 * v);        // even integer nearest v (within 1)
        m.phi = (float)(v - m.I);                   // |phi| <= 1
        if (__builtin_fabs(m.I) < 4194304.0) m.M = (float)(12582912.0 + m.I);   // exact
      }
      ms[a] = m;
    }
  }
}

// Workgroup 0 computes the constants; any others reset a share of the top-k
// state each, at the same time.
constexpr int PREP_RESET_PARTS = 8;

__global__ __launch_bounds__(256) void score_prep_kernel(PrepJob job) {
  if (blockIdx.x > 0) {
    topk_state_reset(job.topk, blockIdx.x - 1, gridDim.x - 1);
    return;
  }
  prep_one(job, false);
}

// Problem blockIdx.x: workgroup y = 0 computes its constants, the others
// reset a share of its top-k state each.
__global__ __launch_bounds__(256) void score_prep_batched_kernel(const PrepJob *__restrict__ jobs, int *counter) {
  // work items of the scoring launch, and of the mixed form's full-chain
  // launch after a queue overflow
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) counter[threadIdx.x] = 0;
  const PrepJob job = load_uniform(jobs + blockIdx.x);
  if (blockIdx.y > 0) {
    if (job.topk) topk_state_reset(job.topk, blockIdx.y - 1, gridDim.y - 1);
    return;
  }
  prep_one(job, false);
}

// Templates per lane: as many FMA chains as the 256 VGPRs of two waves per SIMD
// hold without spilling (a slot costs 2K + 5 registers).
constexpr int tpl_for(int K) {
  const int t = K <= 6 ? 190 / (2 * K + 5) : 180 / (2 * K + 3);
  return t > 16 ? 16 : (t < 1 ? 1 : t);
}
// a smaller tile for the autotuner: about two thirds of the default slots
constexpr int tpl_alt(int K) {
  const int t = tpl_for(K) * 2 / 3;
  return t < 1 ? 1 : t;
}
constexpr bool has_alt(int K) { return K == 8 || K == 16; }
// The standalone kernel: half the 512-thread kernel's slots (rounded up), in
// 1024-thread workgroups.  At K = 8 that is five (the 512-thread kernel held
// a tenth slot at FP32, ~2 % faster than nine); at K = 16 three, which spill
// a few VGPRs in the tile prologue and still measured fastest.
template <int K, typename PT>
constexpr int tpl_fast() {
  constexpr int t512 = (K == 8 && sizeof(PT) == 4) ? 10 : tpl_for(K);
  return (t512 + 1) / 2;
}

template <typename Kern>
hipError_t set_lds(Kern kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <int K, typename PT>
hipError_t launch_fast_k(const ScoreParams &p, int grid, size_t lds, hipStream_t stream) {
  constexpr int TPL = tpl_fast<K, PT>();
  auto kern = score_fast_kernel<K, TPL, PT>;
  hipError_t err = set_lds(kern, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(FAST_THREADS), lds, stream, p);
  return hipGetLastError();
}

template <int K, typename PT>
hipError_t launch_batched_k(const BatchLaunch &b, hipStream_t stream) {
  hipError_t err;
  if constexpr (has_alt(K)) {
    if (b.tpl == tpl_alt(K)) {
      auto kern = score_batched_kernel<K, tpl_alt(K), PT>;
      if ((err = set_lds(kern, b.lds)) != hipSuccess) return err;
      hipLaunchKernelGGL(kern, dim3(b.grid), dim3(SCORE_THREADS), b.lds, stream, b.params, b.items, b.n_items, b.counter);
      return hipGetLastError();
    }
  }
  auto kern = score_batched_kernel<K, tpl_for(K), PT>;
  if ((err = set_lds(kern, b.lds)) != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(b.grid), dim3(SCORE_THREADS), b.lds, stream, b.params, b.items, b.n_items, b.counter);
  return hipGetLastError();
}

template <typename PT, int... Ks>
hipError_t dispatch_fast(int K, const ScoreParams &p, int grid, size_t lds, hipStream_t stream,
                         std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks ? (err = launch_fast_k<Ks, PT>(p, grid, lds, stream), true) : false) || ...);
  return err;
}

template <typename PT, int... Ks>
hipError_t dispatch_batched(int K, const BatchLaunch &b, hipStream_t stream, std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks ? (err = launch_batched_k<Ks, PT>(b, stream), true) : false) || ...);
  return err;
}

template <typename PT>
hipError_t launch_validate(const ScoreParams &p, int K, int grid, size_t lds, hipStream_t stream) {
  auto kern = score_validate_kernel<PT>;
  hipError_t err = set_lds(kern, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(SCORE_THREADS), lds, stream, p, K);
  return hipGetLastError();
}

}  // namespace

int score_templates_per_lane(int K, bool alt) {
  switch (K) {
    case 8: return alt ? tpl_alt(8) : tpl_for(8);
    case 16: return alt ? tpl_alt(16) : tpl_for(16);
    default: return tpl_for(K);
  }
}

hipError_t launch_score_prep(const PrepJob &job, hipStream_t stream) {
  hipLaunchKernelGGL(score_prep_kernel, dim3(job.topk ? 1 + PREP_RESET_PARTS : 1), dim3(256), 0, stream, job);
  return hipGetLastError();
}

hipError_t launch_score_prep_batched(const PrepJob *jobs, int n_jobs, int *counter, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(score_prep_batched_kernel, dim3(n_jobs, 1 + PREP_RESET_PARTS), dim3(256), 0, stream, jobs, counter);
  return hipGetLastError();
}

hipError_t launch_score_batched(const BatchLaunch &b, hipStream_t stream) {
  using Ks = std::make_integer_sequence<int, EMRI_MAX_K + 1>;
  if (b.dtype == EMRI_F32) return dispatch_batched<float>(b.K, b, stream, Ks{});
  return dispatch_batched<__half>(b.K, b, stream, Ks{});
}

hipError_t launch_score(const ScoreParams &p, int K, int dtype, bool validate, int grid, size_t lds,
                        hipStream_t stream) {
  if (validate)
    return dtype == EMRI_F32 ? launch_validate<float>(p, K, grid, lds, stream)
                             : launch_validate<__half>(p, K, grid, lds, stream);
  using Ks = std::make_integer_sequence<int, EMRI_MAX_K + 1>;
  if (dtype == EMRI_F32) return dispatch_fast<float>(K, p, grid, lds, stream, Ks{});
  return dispatch_fast<__half>(K, p, grid, lds, stream, Ks{});
}

}  // namespace emri
