// Mixed-precision form of the scoring kernel: the track contraction
// sum_k c_k (U T)[alpha, k] of Eq. (10) runs on the matrix cores in BF16 with
// FP32 accumulation; the per-segment offset f0 T and the rounding to a bin
// stay in FP64; the power may be stored in FP16.
//
// Split products.  Every FP32 coefficient is the exact sum of three BF16
// pieces c = c0 + c1 + c2 (8 + 8 + 8 significant bits), and every FP64 value
// U T is split the same way into u0 + u1 + u2 (about 24 bits).  The products
// kept are those with piece orders a + b <= 2:
//     c0 u0 + (c0 u1 + c1 u0) + (c0 u2 + c1 u1 + c2 u0),
// six products per coefficient; the dropped ones are below 2^-24 of |c u|, the
// size of the FP32 accumulator's own rounding.  They are accumulated smallest
// first, on top of the fraction phi of f0 T.
//
// Layout on the matrix cores (v_mfma_f32_4x4x4_16b_bf16: 16 blocks of a 4x4x4
// product per wave).  One instruction multiplies the 4 x 4 matrix A (rows = the
// 4 segments of a staging step, columns = 4 coefficients' pieces) by the 4 x 4
// matrix B (4 coefficients' pieces of the block's 4 templates); all 16 blocks
// share A.  Lane l supplies row l%4 of A (segment l%4) and column l%4 of its
// block's B (its own template), and receives that template's 4 segment
// results, one per register: register r holds segment r of the step for every
// lane, so the gathers of one register read one spectrogram row.
//
// Per (template, segment), with D the FP32 contraction started at phi, where
// f0 T = I + phi with I an even integer (FP64) and phi = f0 T - I rounded to
// FP32 (|phi| <= 1):
//     bin = rint(I + D) = I + rint(D)
// (an even I keeps half-to-even ties on the same side), which is one FP32 add
// with the per-segment constant M = 1.5*2^23 + I: the bits of D + M are
// 0x4B400000 + I + rint(D) for |I + D| < 2^22 (templates that could leave
// that range take an FP64 path), so with the bin range [k_min - 1, k_max + 1]
// shifted by 0x4B400000 the same for every segment,
//     address = E * (med3(bits, lo, hi) + B/E - 0x4B400000).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "common.h"
#include "score_internal.h"
#include "staging.h"

namespace emri {
namespace {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kPairs = 6;
// (U piece, c piece) of the six product groups, smallest first
constexpr int pair_u(int p) { return p == 0 ? 2 : (p == 1 ? 1 : (p == 2 ? 0 : (p == 3 ? 1 : 0))); }
constexpr int pair_c(int p) { return p == 0 ? 0 : (p == 1 ? 1 : (p == 2 ? 2 : (p == 3 ? 0 : (p == 4 ? 1 : 0)))); }

// The three BF16 pieces of TPL templates' coefficients, KG groups of 4 each.
template <int KG, int TPL>
struct Pieces {
  short4_t v[TPL][3][KG];
};

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to BF16 (nearest even; one v_cvt_pk_bf16_f32), as
// one dword (a in the low half), and the FP32 values of those halves.
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((float2_t){a, b}, bf16x2_t));
}
__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// Coefficients of template j (zeros if not live), padded to whole groups.
template <int K, int KG>
__device__ __forceinline__ void load_coeffs(const ScoreParams &p, int64_t j, bool live, float (&cf)[4 * KG]) {
#pragma unroll
  for (int k = 0; k < 4 * KG; ++k) cf[k] = 0.0f;
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int k = 0; k < K; k += 4) {
      const float4 v = live ? reinterpret_cast<const float4 *>(p.coeffs + (size_t)j * K)[k / 4]
                            : make_float4(0.f, 0.f, 0.f, 0.f);
      cf[k] = v.x;
      cf[k + 1] = v.y;
      cf[k + 2] = v.z;
      cf[k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) cf[k] = live ? p.coeffs[(size_t)j * K + k] : 0.0f;
  }
}

// The tests of one template from its coefficients and the bounds of prep:
// wild if it could place a track at |x| >= 2^21 bins (huge or non-finite
// values); above K = 8, tail_small if the reduced chain covers it.  The
// reduced launch and the re-scoring of queued tiles take the same decisions
// from the same values.
template <int K, int KG>
__device__ __forceinline__ void template_tests(const float (&cf)[4 * KG], const_dptr bnd, bool &wild,
                                               bool &tail_small) {
  // every operation rounded on its own (no fused multiply-add), so that
  // each inlined copy takes the same decision
#pragma clang fp contract(off)
  // the bound in FP32: K + 1 terms, each rounded at most three times
  // (bound, product, sum), stay within 3 (K + 1) 2^-24 < 1e-5 of the exact
  // sum, so b < 2^21 (1 - 1e-5) implies the exact bound is below 2^21; then
  // |I + D| < 2^22 and the FP32 rounding of D + M is exact
  float b = (float)bnd[0];
  float bg[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) bg[g] = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float t = __builtin_fabsf(cf[k]) * (float)bnd[1 + k];
    b += t;
    bg[k / 4] += t;
  }
  wild = !(b < 2097152.0f * 0.99999f);
  tail_small = true;
  if constexpr (KG >= 3) {
    // the reduced chain's limits, less a margin of 1 % for the FP32
    // rounding of these sums (non-finite values fail the test)
    float all = 0.0f;
#pragma unroll
    for (int g = 0; g < KG; ++g) all += bg[g];
    tail_small = bg[2] <= 0x1p-9f * 0.99f * all;
    if constexpr (KG == 4) tail_small = tail_small && bg[3] <= 0x1p-17f * 0.99f * all;
  }
}

// Load and split the coefficients of this lane's TPL templates of tile t0.
// Returns true if any of them could place a track at |x| >= 2^21 bins (huge
// or non-finite values), from the per-segment bounds of prep.  Above K = 8,
// needs_full is true if any of them needs the full chains (template_tests:
// wild, or not covered by the reduced chain).
template <int K, int KG, int TPL>
__device__ __forceinline__ bool load_pieces(const ScoreParams &p, int64_t t0, int64_t j_end, Pieces<KG, TPL> &pc,
                                            bool &needs_full) {
  const int tid = threadIdx.x;
  const_dptr bnd = (const_dptr)p.bound;
  bool wild = false;
  needs_full = false;
#pragma unroll
  for (int s = 0; s < TPL; ++s) {
    const int64_t j = t0 + (int64_t)s * mixed_threads(K) + tid;
    const bool live = j < j_end;
    float cf[4 * KG];
#pragma unroll
    for (int k = 0; k < 4 * KG; ++k) cf[k] = 0.0f;
    if constexpr (K % 4 == 0) {
#pragma unroll
      for (int k = 0; k < K; k += 4) {
        const float4 v = live ? reinterpret_cast<const float4 *>(p.coeffs + (size_t)j * K)[k / 4]
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        cf[k] = v.x;
        cf[k + 1] = v.y;
        cf[k + 2] = v.z;
        cf[k + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) cf[k] = live ? p.coeffs[(size_t)j * K + k] : 0.0f;
    }
    // the bound in FP32: K + 1 terms, each rounded at most three times
    // (bound, product, sum), stay within 3 (K + 1) 2^-24 < 1e-5 of the exact
    // sum, so b < 2^21 (1 - 1e-5) implies the exact bound is below 2^21; then
    // |I + D| < 2^22 and the FP32 rounding of D + M is exact
    float b = (float)bnd[0];
#pragma unroll
    for (int k = 0; k < K; ++k) b += __builtin_fabsf(cf[k]) * (float)bnd[1 + k];
    wild |= !(b < 2097152.0f * 0.99999f);
    if constexpr (KG >= 3) {
      bool wild_s, tail_small;
      template_tests<K, KG>(cf, bnd, wild_s, tail_small);
      needs_full |= wild_s || !tail_small;
    }
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      // pieces of coefficients 4g .. 4g+3, two per conversion: each remainder
      // is exact in FP32, and the last has at most 8 significant bits
      float r[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] = cf[4 * g + q];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const unsigned w01 = bf16_pair(r[0], r[1]), w23 = bf16_pair(r[2], r[3]);
        pc.v[s][a][g] = __builtin_bit_cast(short4_t, (uint2){w01, w23});
        r[0] -= bf16_lo(w01);
        r[1] -= bf16_hi(w01);
        r[2] -= bf16_lo(w23);
        r[3] -= bf16_hi(w23);
      }
    }
  }
  return wild;
}

// Reduced chain (RED, three or four coefficient groups).  Above K = 8 the
// last groups of an SVD basis carry little: in draws from the one-year box
// the bound sum_k |c_k| max_alpha |U T| of group 2 is at most 1.0e-3 of a
// template's whole bound (K = 9 .. 16), and of group 3 1.6e-6 (K = 16).  The
// reduced chain keeps, for group 2, the products of piece order <= 1
// (c0 u0, c0 u1, c1 u0) and, for group 3, c0 u0 alone.  Piece i of a value
// is at most 2^-8i of it, so the terms left out are at most ~3 * 2^-16
// (group 2) and ~2^-7 (group 3) of the group's bound; for a template whose
// group bounds are at most 2^-9 and 2^-17 of its whole bound (tail_small)
// they move a position by at most ~2.5 * 2^-24 of that bound (~1.5 * 2^-24
// with three groups), against up to 18 or 24 roundings of 2^-24 of their
// partial sums in the full chains' FP32 accumulation.  A wave of the reduced
// launch that holds a template outside those limits (or a wild one) queues
// its tile, and a second launch scores the queued tiles again with the full
// chains, which write the statistics of the templates that need them.
template <int KG, bool RED>
constexpr bool product_kept(int i) {
  const int p = i / KG, g = i % KG;            // pair (smallest first) and group
  return !RED || !((g == 2 && p < 3) || (g == 3 && p < 5));
}
template <int KG, bool RED>
constexpr int products_in_part(int part) {
  constexpr int NI = kPairs * KG;
  int n = 0;
  for (int i = part * NI / 4; i < (part + 1) * NI / 4; ++i) n += product_kept<KG, RED>(i) ? 1 : 0;
  return n;
}

// Part PART of 4 of the matrix products of one staging step: instructions
// [PART*NI/4, (PART+1)*NI/4) of every slot's chain (NI = 6*KG, smallest
// products first; with RED the products above are left out); the chains
// start from phi.
template <int KG, int TPL, int PART, bool RED>
__device__ __forceinline__ void products_part(const short4_t (&ua)[3][KG], const float4_t &phi,
                                              const Pieces<KG, TPL> &pc, float4_t (&d)[TPL]) {
  constexpr int NI = kPairs * KG;
  static_assert(product_kept<KG, RED>(0), "every chain starts from phi");
#pragma unroll
  for (int i = PART * NI / 4; i < (PART + 1) * NI / 4; ++i) {
    if (!product_kept<KG, RED>(i)) continue;
#pragma unroll
    for (int s = 0; s < TPL; ++s)
      d[s] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ua[pair_u(i / KG)][i % KG], pc.v[s][pair_c(i / KG)][i % KG],
                                                    i == 0 ? phi : d[s], 0, 0, 0);
  }
}

template <int KG, int TPL, bool RED>
__device__ __forceinline__ void step_products(const short4_t (&ua)[3][KG], const float4_t &phi,
                                              const Pieces<KG, TPL> &pc, float4_t (&d)[TPL]) {
  products_part<KG, TPL, 0, RED>(ua, phi, pc, d);
  products_part<KG, TPL, 1, RED>(ua, phi, pc, d);
  products_part<KG, TPL, 2, RED>(ua, phi, pc, d);
  products_part<KG, TPL, 3, RED>(ua, phi, pc, d);
}

// Operands of the products of one staging step r0: the A rows (segment
// r0 + lane % 4), the fractions phi of f0 T (the chains' start) and the
// integer offsets I.
// Clamp bounds of the FP32 rounding path (wave-uniform; hi in a VGPR, as the
// clamp instruction reads at most one scalar operand).
struct BinClamp {
  int lo, hi;
};

template <int KG>
struct StepOps {
  short4_t ua[3][KG];
  float4_t phi;
  double I[4];      // the FP64 path's offsets
  float M[4];       // 1.5*2^23 + I (the FP32 rounding path)
};

// Issue the loads of step r0's operands (the table rows from LDS, the
// per-segment values with scalar loads); the caller waits for them.
template <int KG>
__device__ __forceinline__ void issue_operands(const unsigned char *tab, const MixedSeg *ms, int r0, StepOps<KG> &op) {
  const int lane = (int)(threadIdx.x & 63);
  const short4_t *row = reinterpret_cast<const short4_t *>(tab + (size_t)(r0 + (lane & 3)) * (3 * KG * 8));
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int g = 0; g < KG; ++g) op.ua[a][g] = row[a * KG + g];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const MixedSeg m = load_uniform(ms + r0 + r);
    op.I[r] = m.I;
    op.M[r] = m.M;
    op.phi[r] = m.phi;
  }
}

// Keep the scalar loads of issue_operands ahead of this point (their results
// are needed here), so that none is outstanding in the next counted waits.
template <int KG>
__device__ __forceinline__ void operands_landed(const StepOps<KG> &op) {
#pragma unroll
  for (int r = 0; r < 4; ++r) asm volatile("" ::"s"(op.I[r]), "s"(op.M[r]));
}

// Interleave the matrix products just issued with the vector work of the same
// scheduling region: one product, then one vector instruction, N times
// (measured: 1.3 % faster at K = 16 than two, no change at K = 8).
template <int N>
__device__ __forceinline__ void interleave_products() {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
    __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);   // one VALU
  }
}

// One staging step r0 (4 segments) with the products dc of this step, while
// the products dn of the next step are issued a quarter per segment,
// interleaved with the address arithmetic, from the operands op loaded during
// the previous step.  The gathers of segment r are in flight while the
// addresses of segment r+1 are computed; the operands of the step after next
// load while the last gathers are in flight.  Segments past n_seg (last step)
// gather in-bounds stale data that is not added.  GUARD: this step may reach
// past n_seg (the last step; others add without a test); FOLD: the FP32 run
// ends here and is added into the FP64 sums (every second step, and the last).
template <int KG, int TPL, typename PT, bool WILD, bool RED, bool GUARD, bool FOLD>
__device__ __forceinline__ void mixed_step(const ScoreParams &p, const Pipe &pp, const unsigned char *tab,
                                           unsigned char *lds, const Pieces<KG, TPL> &pc, int r0, int half,
                                           const float4_t (&dc)[TPL], const double (&Ic)[4], const float (&Mc)[4],
                                           float4_t (&dn)[TPL], double (&In)[4], float (&Mn)[4], StepOps<KG> &op,
                                           const BinClamp &bcl, float (&acc)[TPL],
                                           double (&sum)[TPL]) {
  constexpr int E = Elem<PT>::bytes;
  static_assert(TPL < 16, "lgkmcnt holds at most 15 outstanding gathers");
  if (pp.wave < SCORE_WAVES) pipe_issue(p, pp, lds, r0 + 4, half ^ 1);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    In[r] = op.I[r];
    Mn[r] = op.M[r];
  }
  __builtin_amdgcn_sched_barrier(0);
  // Gathers of DEPTH segments in flight: those of segment r are issued before
  // waiting for those of segment r - DEPTH (lgkmcnt(DEPTH * TPL): only LDS
  // reads are outstanding here, and lgkmcnt counts at most 15).  Two pay up
  // to K = 8 (1 % at K = 8); at K = 16 the spilling kernel is 0.3 % slower.
  constexpr int DEPTH = (KG <= 2 && 2 * TPL < 16) ? 2 : 1;
  constexpr int NV = DEPTH + 1;
  typename Elem<PT>::raw_t v[NV][TPL];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const BufConst bc = buffer_consts<PT>(p, lds, half, r);
    // bits(D + M) = 0x4B400000 + I + rint(D) = 0x4B400000 + bin for |I + D| < 2^22
    // (M = 1.5*2^23 + I; I even keeps ties even); clamped in that shifted
    // range, the bin's LDS element is it plus cr = base - 0x4B400000
    const int cr = bc.base - 0x4B400000;
    int addr[TPL];
#pragma unroll
    for (int s = 0; s < TPL; ++s) {
      if constexpr (WILD) {
        const double x = (double)dc[s][r] + Ic[r];
        const double y = (__builtin_fabs(x) < kWildLimit) ? x + bc.magic : bc.magic - 2.0;
        addr[s] = E * clamp_i32(low_word(y), bc.lo, bc.hi);
      } else {
        const int bits = __float_as_int(dc[s][r] + Mc[r]);
        addr[s] = E * (clamp_i32(bits, bcl.lo, bcl.hi) + cr);
      }
    }
    if constexpr (KG <= 2) {
      // up to K = 8 the gathers go out before this quarter's products, which
      // then run while they are in flight (measured: K = 8 9.93 -> 9.77 ms,
      // batched 10.32 -> 10.10 ms; K = 16 3 % slower, so it keeps the order
      // below, with the products interleaved with the address arithmetic)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < TPL; ++s) v[r % NV][s] = Elem<PT>::raw(addr[s]);
      __builtin_amdgcn_sched_barrier(0);
      if (r == 0) products_part<KG, TPL, 0, RED>(op.ua, op.phi, pc, dn);
      if (r == 1) products_part<KG, TPL, 1, RED>(op.ua, op.phi, pc, dn);
      if (r == 2) products_part<KG, TPL, 2, RED>(op.ua, op.phi, pc, dn);
      if (r == 3) products_part<KG, TPL, 3, RED>(op.ua, op.phi, pc, dn);
      __builtin_amdgcn_sched_barrier(0);
    } else {
      // each quarter's products interleaved one for one with the vector work
      if (r == 0) {
        products_part<KG, TPL, 0, RED>(op.ua, op.phi, pc, dn);
        interleave_products<products_in_part<KG, RED>(0) * TPL>();
      }
      if (r == 1) {
        products_part<KG, TPL, 1, RED>(op.ua, op.phi, pc, dn);
        interleave_products<products_in_part<KG, RED>(1) * TPL>();
      }
      if (r == 2) {
        products_part<KG, TPL, 2, RED>(op.ua, op.phi, pc, dn);
        interleave_products<products_in_part<KG, RED>(2) * TPL>();
      }
      if (r == 3) {
        products_part<KG, TPL, 3, RED>(op.ua, op.phi, pc, dn);
        interleave_products<products_in_part<KG, RED>(3) * TPL>();
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < TPL; ++s) v[r % NV][s] = Elem<PT>::raw(addr[s]);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (r >= DEPTH) {
      __builtin_amdgcn_s_waitcnt(0xC07F | ((DEPTH * TPL) << 8));   // gathers of segment r - DEPTH
      __builtin_amdgcn_sched_barrier(0);
      if (!GUARD || r0 + r - DEPTH < p.n_seg) {
#pragma unroll
        for (int s = 0; s < TPL; ++s) acc[s] = Elem<PT>::add(acc[s], v[(r - DEPTH) % NV][s], p.one);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if constexpr (DEPTH == 2) {
    __builtin_amdgcn_s_waitcnt(0xC07F | (TPL << 8));             // gathers of segment 2
    __builtin_amdgcn_sched_barrier(0);
    if (!GUARD || r0 + 2 < p.n_seg) {
#pragma unroll
      for (int s = 0; s < TPL; ++s) acc[s] = Elem<PT>::add(acc[s], v[2][s], p.one);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // operands of step r0 + 8 (any step in range past the end: loaded, unused)
  const int rn = r0 + 8 < p.n_seg ? r0 + 8 : r0;
  issue_operands<KG>(tab, reinterpret_cast<const MixedSeg *>(p.mseg), rn, op);
  __builtin_amdgcn_s_waitcnt(0xC07F);          // the last gathers and the operands
  operands_landed<KG>(op);
  __builtin_amdgcn_sched_barrier(0);
  if (!GUARD || r0 + 3 < p.n_seg) {
#pragma unroll
    for (int s = 0; s < TPL; ++s) acc[s] = Elem<PT>::add(acc[s], v[3 % NV][s], p.one);
  }
  // FP32 runs of 8 segments (two steps), then FP64, as in the plain kernel
  if constexpr (FOLD) {
#pragma unroll
    for (int s = 0; s < TPL; ++s) {
      sum[s] += (double)acc[s];
      acc[s] = 0.0f;
    }
  }
  pipe_publish<PT>(p, pp, lds, half ^ 1);
}

// One tile: TPL slots of mixed_threads(K) templates against every segment.  Software
// pipelined: while a wave gathers with the products of step n it also issues
// the matrix products of step n+1 (two steps per loop turn, so the two product
// buffers swap roles without copies).  Above K = 8 the caller has queued the
// first rows' copies (`queued`).
template <int KG, int TPL, typename PT, bool WILD, bool RED>
__device__ __forceinline__ void run_tile_mixed(const ScoreParams &p, const Pipe *queued, unsigned char *tab,
                                               unsigned char *lds, const Pieces<KG, TPL> &pc, double (&sum)[TPL]) {
  float acc[TPL];
#pragma unroll
  for (int s = 0; s < TPL; ++s) acc[s] = 0.0f;
  Pipe pp;
  if constexpr (KG > 2) {
    pp = *queued;
  } else {
    pp = pipe_init<PT>(p);
    if (pp.wave < SCORE_WAVES) pipe_issue(p, pp, lds, 0, 0);
  }
  pipe_publish<PT>(p, pp, lds, 0);
  float4_t da[TPL], db[TPL];
  double Ia[4], Ib[4];
  float Ma[4], Mb[4];
  // the bin range [k_min - 1, k_max + 1] in the shifted integer domain of the
  // FP32 rounding, the upper bound held in a vector register for the tile
  BinClamp bcl;
  bcl.lo = p.k_min - 1 + 0x4B400000;
  asm volatile("v_mov_b32 %0, %1" : "=v"(bcl.hi) : "s"(p.k_max + 1 + 0x4B400000));
  StepOps<KG> op;
  if (p.n_seg > 0) {
    const MixedSeg *ms = reinterpret_cast<const MixedSeg *>(p.mseg);
    issue_operands<KG>(tab, ms, 0, op);
    step_products<KG, TPL, RED>(op.ua, op.phi, pc, da);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Ia[r] = op.I[r];
      Ma[r] = op.M[r];
    }
    issue_operands<KG>(tab, ms, p.n_seg > 4 ? 4 : 0, op);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    operands_landed<KG>(op);
    __builtin_amdgcn_sched_barrier(0);
  }
  // whole pairs of steps, then the last one or two steps (1 to 7 segments)
  int r0 = 0;
  for (; r0 + 8 <= p.n_seg; r0 += 8) {
    mixed_step<KG, TPL, PT, WILD, RED, false, false>(p, pp, tab, lds, pc, r0, 0, da, Ia, Ma, db, Ib, Mb, op, bcl, acc, sum);
    mixed_step<KG, TPL, PT, WILD, RED, false, true>(p, pp, tab, lds, pc, r0 + 4, 1, db, Ib, Mb, da, Ia, Ma, op, bcl, acc, sum);
  }
  if (r0 + 4 < p.n_seg) {
    mixed_step<KG, TPL, PT, WILD, RED, false, false>(p, pp, tab, lds, pc, r0, 0, da, Ia, Ma, db, Ib, Mb, op, bcl, acc, sum);
    mixed_step<KG, TPL, PT, WILD, RED, true, true>(p, pp, tab, lds, pc, r0 + 4, 1, db, Ib, Mb, da, Ia, Ma, op, bcl, acc, sum);
  } else if (r0 < p.n_seg) {
    mixed_step<KG, TPL, PT, WILD, RED, true, true>(p, pp, tab, lds, pc, r0, 0, da, Ia, Ma, db, Ib, Mb, op, bcl, acc, sum);
  }
}

// Copy the piece table of a stream into the front of LDS (before the staging halves).
template <int NT>
__device__ __forceinline__ void load_table(const ScoreParams &p, unsigned char *tab) {
  const int n16 = p.mtab_bytes >> 4;
  const uint4 *src = reinterpret_cast<const uint4 *>(p.mtab);
  uint4 *dst = reinterpret_cast<uint4 *>(tab);
  for (int i = threadIdx.x; i < n16; i += NT) dst[i] = src[i];
}

__device__ __forceinline__ unsigned char *staging_base(const ScoreParams &p, unsigned char *lds) {
  return lds + ((p.mtab_bytes + 1023) & ~1023);
}

// RED: the reduced chain, queueing the tile when a template needs the full
// ones; ONLY_FULL: the full chains, writing only the statistics of the
// templates that need them (the re-scoring of queued tiles), so that every
// statistic depends on its own template alone, not on its tile-mates.
template <int K, int T, typename PT, bool RED, bool ONLY_FULL = false>
__device__ __forceinline__ void score_tile_mixed(const ScoreParams &p, unsigned char *lds, unsigned char *stage,
                                                 int64_t t0, int64_t j_end) {
  constexpr int KG = (K + 3) / 4;
  // Above K = 8 the first rows' copies are queued before the coefficient
  // loads, so that both are in flight together (the previous tile's last
  // barrier has retired every read of the staging halves): measured 2.6 %
  // faster at K = 16, but 2 % slower at K = 8 and 3 % slower in the plain
  // batched kernel, where they follow the coefficients.
  Pipe pp{};
  if constexpr (KG > 2) {
    pp = pipe_init<PT>(p);
    if (pp.wave < SCORE_WAVES) pipe_issue(p, pp, stage, 0, 0);
  }
  Pieces<KG, T> pc;
  bool needs_full;
  const bool wild = load_pieces<K, KG, T>(p, t0, j_end, pc, needs_full);
  double sum[T];
#pragma unroll
  for (int s = 0; s < T; ++s) sum[s] = 0.0;
  if constexpr (RED) {
    // one chain only: a wave holding a template it does not cover queues the
    // tile for the full chains (waves of one tile may queue it more than once;
    // the full chains then write the same values again)
    if (__any(needs_full) && (threadIdx.x & 63) == 0) {
      const unsigned e = atomicAdd(p.redo, 1u);
      const int64_t t_end = t0 + (int64_t)T * mixed_threads(K) < j_end ? t0 + (int64_t)T * mixed_threads(K) : j_end;
      if (e < (unsigned)MIXED_REDO_CAP)
        reinterpret_cast<uint4 *>(p.redo + 4)[e] = make_uint4((unsigned)t0, (unsigned)t_end, p.redo_tag, 0u);
    }
    run_tile_mixed<KG, T, PT, false, true>(p, &pp, lds, stage, pc, sum);
  } else if (__any(wild)) {
    run_tile_mixed<KG, T, PT, true, false>(p, &pp, lds, stage, pc, sum);
  } else {
    run_tile_mixed<KG, T, PT, false, false>(p, &pp, lds, stage, pc, sum);
  }
#pragma unroll
  for (int s = 0; s < T; ++s) {
    const int64_t j = t0 + (int64_t)s * mixed_threads(K) + threadIdx.x;
    bool write = j < j_end;
    if constexpr (ONLY_FULL) {
      // the template's tests again (its coefficients are read once more,
      // rather than a mask kept live through the tile)
      float cf[4 * KG];
      load_coeffs<K, KG>(p, j, write, cf);
      bool wild_s, tail_small;
      template_tests<K, KG>(cf, (const_dptr)p.bound, wild_s, tail_small);
      write = write && (wild_s || !tail_small);
    }
    if (write) p.stat[j] = (float)sum[s];
  }
}

// Tiles of TPL slots; a last tile that fits in half as many slots runs with half.
template <int K, int TPL, typename PT, bool RED = false, bool ONLY_FULL = false>
__device__ __forceinline__ void score_range_mixed(const ScoreParams &p, unsigned char *lds, int64_t j_begin,
                                                  int64_t j_end) {
  constexpr int TAIL = (TPL + 1) / 2;
  unsigned char *stage = staging_base(p, lds);
  constexpr int NT = mixed_threads(K);
  for (int64_t t0 = j_begin; t0 < j_end; t0 += (int64_t)TPL * NT) {
    if (TAIL < TPL && j_end - t0 <= (int64_t)TAIL * NT) {
      score_tile_mixed<K, TAIL, PT, RED, ONLY_FULL>(p, lds, stage, t0, j_end);
      break;
    }
    score_tile_mixed<K, TPL, PT, RED, ONLY_FULL>(p, lds, stage, t0, j_end);
  }
}

// MODE 0: the full chains over the workgroup's range; MODE 1: the reduced
// chain (queues the tiles it does not cover in p.redo); MODE 2: the full
// chains over the tiles the reduced launch queued (grid-strided; nothing if
// the queue overflowed); MODE 3: the full chains over the workgroup's range
// if the queue overflowed (nothing otherwise).  Modes 2 and 3 write only the
// statistics of the templates that need the full chains.
template <int K, int TPL, typename PT, int MODE>
__global__ __launch_bounds__(mixed_threads(K)) void score_mixed_kernel(ScoreParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  if constexpr (MODE >= 2) {
    const unsigned n_redo = __builtin_amdgcn_readfirstlane(*(volatile unsigned *)p.redo);
    if (MODE == 3 ? n_redo <= (unsigned)MIXED_REDO_CAP : (n_redo > (unsigned)MIXED_REDO_CAP || blockIdx.x >= n_redo))
      return;
    if constexpr (MODE == 2) {
      load_table<mixed_threads(K)>(p, lds);
      init_lds(p, staging_base(p, lds));
      const uint4 *q = reinterpret_cast<const uint4 *>(p.redo + 4);
      for (unsigned e = blockIdx.x; e < n_redo; e += gridDim.x) {
        const uint4 t = q[e];
        score_tile_mixed<K, TPL, PT, false, true>(p, lds, staging_base(p, lds), (int64_t)t.x, (int64_t)t.y);
      }
      return;
    }
  }
  load_table<mixed_threads(K)>(p, lds);
  init_lds(p, staging_base(p, lds));
  const int64_t j_begin = (int64_t)blockIdx.x * p.per_block;
  const int64_t j_end = j_begin + p.per_block < p.n_tmpl ? j_begin + p.per_block : p.n_tmpl;
  score_range_mixed<K, TPL, PT, MODE == 1, MODE == 3>(p, lds, j_begin, j_end);
}

// Batched form of the mixed kernel (work items claimed as in the plain
// batched kernel; the piece table is reloaded when the stream changes).
// MODE as in score_mixed_kernel: 0 the full chains, 1 the reduced chain
// (queueing tiles tagged with their problem), 3 the full chains over every
// item, writing only the templates that need them, if the queue overflowed
// (claims from counter[1]; nothing otherwise).
template <int K, int TPL, typename PT, int MODE>
__global__ __launch_bounds__(mixed_threads(K)) void score_mixed_batched_kernel(const ScoreParams *__restrict__ params,
                                                                            const BatchItem *__restrict__ items,
                                                                            int n_items, int *counter,
                                                                            const unsigned *redo) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ int slot;
  if constexpr (MODE == 3) {
    if (__builtin_amdgcn_readfirstlane(*(const volatile unsigned *)redo) <= (unsigned)MIXED_REDO_CAP) return;
    counter += 1;
  }
  int table_of = -1;
  for (;;) {
    const int it = claim_item(counter, &slot);
    if (it >= n_items) break;
    const BatchItem item = load_uniform(items + it);
    const ScoreParams p = load_uniform(params + item.stream);
    if (item.stream != table_of) {     // claim_item's barriers order this after the last reads
      load_table<mixed_threads(K)>(p, lds);
      table_of = item.stream;
    }
    init_lds(p, staging_base(p, lds));
    score_range_mixed<K, TPL, PT, MODE == 1, MODE == 3>(p, lds, item.begin, item.end);
  }
}

// The queued tiles of a batched reduced-chain launch, with the full chains
// (each entry names its problem; grid-strided; nothing if the queue
// overflowed), writing only the templates that need them.
template <int K, int TPL, typename PT>
__global__ __launch_bounds__(mixed_threads(K)) void score_mixed_requeue_kernel(const ScoreParams *__restrict__ params,
                                                                            const unsigned *redo) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const unsigned n_redo = __builtin_amdgcn_readfirstlane(*(const volatile unsigned *)redo);
  if (n_redo > (unsigned)MIXED_REDO_CAP || blockIdx.x >= n_redo) return;
  const uint4 *q = reinterpret_cast<const uint4 *>(redo + 4);
  int table_of = -1;
  for (unsigned e = blockIdx.x; e < n_redo; e += gridDim.x) {
    const uint4 t = q[e];
    const ScoreParams p = load_uniform(params + t.z);
    __syncthreads();                   // every wave is done with the previous tile's LDS
    if ((int)t.z != table_of) {
      load_table<mixed_threads(K)>(p, lds);
      table_of = (int)t.z;
    }
    init_lds(p, staging_base(p, lds));
    score_tile_mixed<K, TPL, PT, false, true>(p, lds, staging_base(p, lds), (int64_t)t.x, (int64_t)t.y);
  }
}

// Templates per lane: up to K = 8 in 1024-thread workgroups (128 VGPRs per
// wave at four waves per SIMD; a tile is as large as with 512 threads and
// twice the templates per lane, but a SIMD has twice the waves to hide the
// latency of the gathers and the matrix products behind: one-year, 1e8
// templates, K = 8 9.51 -> 8.39 ms, K = 16 16.14 -> 14.99 ms), above in
// 768-thread workgroups with three templates per lane (K = 16 12.95 -> 12.39
// ms against two per lane at 1024 threads; at K = 8 four per lane at 768
// threads measured the same as three at 1024).
constexpr int mixed_tpl(int K) { return K <= 4 ? 4 : 3; }

template <typename Kern>
hipError_t set_lds(Kern kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <int K, typename PT, int MODE>
hipError_t launch_mixed_mode(const ScoreParams &p, int grid, size_t lds, hipStream_t stream) {
  auto kern = score_mixed_kernel<K, mixed_tpl(K), PT, MODE>;
  hipError_t err = set_lds(kern, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(mixed_threads(K)), lds, stream, p);
  return hipGetLastError();
}

// Above K = 8 (with a tile queue in p.redo, whose count the prep kernel of
// the call cleared): the reduced launch, then the full chains over the tiles
// it queued (workgroups past the queue's length return at once), then over
// the whole batch only if the queue overflowed.
template <int K, typename PT>
hipError_t launch_mixed_k(const ScoreParams &p, int grid, size_t lds, hipStream_t stream) {
  if constexpr (mixed_groups(K) >= 3) {
    if (p.redo) {
      hipError_t err = launch_mixed_mode<K, PT, 1>(p, grid, lds, stream);
      if (err == hipSuccess) err = launch_mixed_mode<K, PT, 2>(p, grid, lds, stream);
      if (err == hipSuccess) err = launch_mixed_mode<K, PT, 3>(p, grid, lds, stream);
      return err;
    }
  }
  return launch_mixed_mode<K, PT, 0>(p, grid, lds, stream);
}

template <int K, typename PT, int MODE>
hipError_t launch_mixed_batched_mode(const BatchLaunch &b, hipStream_t stream) {
  auto kern = score_mixed_batched_kernel<K, mixed_tpl(K), PT, MODE>;
  hipError_t err = set_lds(kern, b.lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(b.grid), dim3(mixed_threads(K)), b.lds, stream, b.params, b.items, b.n_items, b.counter,
                     (const unsigned *)b.redo);
  return hipGetLastError();
}

// Above K = 8 (with a tile queue in b.redo, whose count the prep kernel of
// the run cleared): the reduced chain over every item, the full chains over
// the queued tiles, then over every item only if the queue overflowed.
template <int K, typename PT>
hipError_t launch_mixed_batched_k(const BatchLaunch &b, hipStream_t stream) {
  if constexpr (mixed_groups(K) >= 3) {
    if (b.redo) {
      hipError_t err = launch_mixed_batched_mode<K, PT, 1>(b, stream);
      if (err == hipSuccess) {
        auto kern = score_mixed_requeue_kernel<K, mixed_tpl(K), PT>;
        err = set_lds(kern, b.lds);
        if (err == hipSuccess) {
          hipLaunchKernelGGL(kern, dim3(b.grid), dim3(mixed_threads(K)), b.lds, stream, b.params,
                             (const unsigned *)b.redo);
          err = hipGetLastError();
        }
      }
      if (err == hipSuccess) err = launch_mixed_batched_mode<K, PT, 3>(b, stream);
      return err;
    }
  }
  return launch_mixed_batched_mode<K, PT, 0>(b, stream);
}

template <typename PT, int... Ks>
hipError_t dispatch_mixed(int K, const ScoreParams &p, int grid, size_t lds, hipStream_t stream,
                          std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks + 1 ? (err = launch_mixed_k<Ks + 1, PT>(p, grid, lds, stream), true) : false) || ...);
  return err;
}

template <typename PT, int... Ks>
hipError_t dispatch_mixed_batched(int K, const BatchLaunch &b, hipStream_t stream, std::integer_sequence<int, Ks...>) {
  hipError_t err = hipErrorInvalidValue;
  ((K == Ks + 1 ? (err = launch_mixed_batched_k<Ks + 1, PT>(b, stream), true) : false) || ...);
  return err;
}

}  // namespace

int mixed_templates_per_lane(int K) { return mixed_tpl(K); }
int mixed_tile_templates(int K) { return mixed_tpl(K) * mixed_threads(K); }

hipError_t launch_score_mixed(const ScoreParams &p, int K, int dtype, int grid, size_t lds, hipStream_t stream) {
  using Ks = std::make_integer_sequence<int, MIXED_MAX_K>;
  if (dtype == EMRI_F32) return dispatch_mixed<float>(K, p, grid, lds, stream, Ks{});
  return dispatch_mixed<__half>(K, p, grid, lds, stream, Ks{});
}

hipError_t launch_score_mixed_batched(const BatchLaunch &b, hipStream_t stream) {
  using Ks = std::make_integer_sequence<int, MIXED_MAX_K>;
  if (b.dtype == EMRI_F32) return dispatch_mixed_batched<float>(b.K, b, stream, Ks{});
  return dispatch_mixed_batched<__half>(b.K, b, stream, Ks{});
}

}  // namespace emri
