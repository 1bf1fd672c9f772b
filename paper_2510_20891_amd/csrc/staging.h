// Device helpers shared by the scoring kernels: LDS element access, the
// rounding / clamping step, and the pipeline that stages spectrogram rows from
// HBM into LDS (layout described in score_internal.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "score_internal.h"

namespace emri {
namespace {

constexpr double kWildLimit = 67108864.0;      // 2^26 bins
constexpr double kNearTie = 1e-6;
constexpr int kLeadIn = SCORE_LDS_LEAD;          // bytes before bin 0 in each LDS buffer

typedef const __attribute__((address_space(4))) double *const_dptr;

typedef __attribute__((address_space(3))) unsigned char lds_byte;

// LDS byte address of a pointer into dynamic shared memory.
__device__ __forceinline__ int lds_address(const void *p) { return (int)(size_t)(const lds_byte *)p; }

// Power elements in LDS.  raw() is the gathered element as stored; add()
// widens it into an FP32 accumulator (for FP16 one v_fma_mix_f32: the product
// with 1.0 is exact, so the result is the rounded sum acc + P).
template <typename PT>
struct Elem;
template <>
struct Elem<float> {
  static constexpr int bytes = 4;
  typedef float raw_t;
  __device__ static float raw(int addr) { return *(const __attribute__((address_space(3))) float *)(size_t)addr; }
  __device__ static float add(float acc, float v, float) { return acc + v; }
  __device__ static float load(int addr) { return raw(addr); }
  __device__ static void zero(int addr) { *(__attribute__((address_space(3))) float *)(size_t)addr = 0.0f; }
};
template <>
struct Elem<__half> {
  static constexpr int bytes = 2;
  typedef _Float16 raw_t;
  __device__ static _Float16 raw(int addr) {
    return __builtin_bit_cast(_Float16, *(const __attribute__((address_space(3))) unsigned short *)(size_t)addr);
  }
  __device__ static float add(float acc, _Float16 v, float one) { return __builtin_fmaf((float)v, one, acc); }
  __device__ static float load(int addr) { return (float)raw(addr); }
  __device__ static void zero(int addr) {
    *(__attribute__((address_space(3))) unsigned short *)(size_t)addr = (unsigned short)0;
  }
};

// med3 of three signed integers in one VALU instruction (lo in an SGPR, hi in a VGPR).
__device__ __forceinline__ int clamp_i32(int x, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "s"(lo), "v"(hi));
  return r;
}

// Per-buffer constants of the rounding / addressing step (in elements).
struct BufConst {
  double magic;
  int lo, hi;
  int base;      // LDS element index (address / E) of bin 0
};

// Row buffer b of LDS half `half`: bin 0 sits pitch_bytes * b after the half's lead-in.
template <typename PT>
__device__ __forceinline__ BufConst buffer_consts(const ScoreParams &p, const unsigned char *lds, int half, int b) {
  constexpr int E = Elem<PT>::bytes;
  // absolute LDS byte address of bin 0, in elements (even: 16-byte aligned)
  const int base = (int)(((unsigned)lds_address(lds) + (unsigned)(half * p.half_bytes + kLeadIn + b * p.pitch_bytes)) / E);
  BufConst bc;
  bc.base = base;
  bc.magic = 6755399441055744.0 + (double)base;     // 1.5*2^52 + base
  bc.lo = base + p.k_min - 1;
  bc.hi = base + p.k_max + 1;
  return bc;
}

__device__ __forceinline__ int low_word(double y) { return (int)(unsigned)__double2loint(y); }

// Wave index as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Staging pipeline.  A step stages G consecutive rows into one LDS half while
// the other half is gathered from; it ends with a wait for this wave's copies,
// the re-zeroing of the zero slots this wave's copies overwrote, and a
// workgroup barrier.  The G rows are one contiguous block in HBM and in LDS, so
// wave w copies its 1 KB chunks w, w+8, w+16, ... with one instruction each.
struct Pipe {
  int wave;
  int lane_off;      // lane * 16: this lane's bytes within a chunk
  int slot_off;      // byte offset (from the half's start) of this lane's zero slot
  bool slot_mine;    // this lane re-zeroes slot_off after each copy
};

template <typename PT>
__device__ __forceinline__ Pipe pipe_init(const ScoreParams &p) {
  constexpr int E = Elem<PT>::bytes;
  Pipe pp;
  pp.wave = wave_id();
  const int lane = (int)(threadIdx.x & 63);
  pp.lane_off = lane * 16;
  pp.slot_mine = false;
  pp.slot_off = 0;
  if (lane < 2 * p.G) {
    pp.slot_off = kLeadIn + zero_slot_rel(lane, p.pitch_bytes, E, p.k_min, p.k_max);
    pp.slot_mine = (int)((p.slot_owner >> (8 * lane)) & 0xffu) == pp.wave;
  }
  return pp;
}

// Queue the copies of rows [r0, r0 + G) (clipped to n_seg) into half `half`.
// The final chunk's lanes that would read past the block re-read its last 16
// bytes; what they write lands in the half's slack, which no gather reads.
__device__ __forceinline__ void pipe_issue(const ScoreParams &p, const Pipe &pp, unsigned char *lds, int r0,
                                           int half) {
  const int rows = step_rows(p.n_seg, r0, p.G);
  if (rows == 0) return;
  const char *src = reinterpret_cast<const char *>(p.power) + (size_t)r0 * (size_t)p.pitch_bytes;
  unsigned char *dst = lds + half * p.half_bytes + kLeadIn;
  for_each_copy(pp.wave, pp.lane_off, rows * p.pitch_bytes, [&](int c, int src_off) {
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src + src_off),
                                     (__attribute__((address_space(3))) void *)(dst + c * STAGE_CHUNK), 16, 0, 0);
  });
}

// Wait for this wave's copies, re-zero the slots they overwrote in half `half`,
// and publish the rows to the workgroup.
template <typename PT>
__device__ __forceinline__ void pipe_publish(const ScoreParams &p, const Pipe &pp, unsigned char *lds, int half) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  if (pp.slot_mine) Elem<PT>::zero(lds_address(lds) + half * p.half_bytes + pp.slot_off);
  __syncthreads();
}

// Zero the three 16-byte areas no copy writes: the lead-in of each half (the
// slot below bin 0 of its first row) and the tail after the second half.
__device__ __forceinline__ void init_lds(const ScoreParams &p, unsigned char *lds) {
  if (threadIdx.x < 3 * kLeadIn) lds[(threadIdx.x / kLeadIn) * p.half_bytes + threadIdx.x % kLeadIn] = 0;
}

// Next work item of a dynamically scheduled launch: one atomic per workgroup,
// broadcast through `slot` (LDS); wave-uniform result.
__device__ __forceinline__ int claim_item(int *counter, int *slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  const int it = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();             // every wave has read the slot before it is reused
  return it;
}

// BF16 with round-to-nearest-even from FP32 (NaN stays NaN), and back.
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

}  // namespace
}  // namespace emri
