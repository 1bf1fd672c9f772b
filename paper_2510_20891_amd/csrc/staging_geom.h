// Geometry of the LDS row staging used by the scoring kernels, as plain C++
// with no HIP dependency: the device pipeline (staging.h) and the host-side
// layout code both use these functions, and a host program can run the same
// arithmetic to check every copy against its buffers.
//
// LDS holds two halves, each a 16-byte lead-in followed by G consecutive
// spectrogram rows exactly as they lie in HBM (pitch_bytes apart), padded up
// to a whole number of 1 KB chunks; a 16-byte tail follows the second half.
// The G rows of a step are one contiguous block of bytes in HBM, copied in
// 1 KB chunks: wave w issues chunks w, w + SCORE_WAVES, ... with one
// 64-lane x 16-byte instruction each.  In the final chunk, lanes that would
// read past the block re-read its last 16 bytes; a lane's LDS destination is
// fixed by its lane index, so those lanes write into the half's slack.
// Zero slot j (j < 2G) belongs to row buffer j/2: the bin just below k_min (j
// even) or just above k_max (j odd).  A copy may overwrite a slot that lies
// inside the copied chunks; the wave that copied that chunk writes the zero
// back after its own copies have landed.
#pragma once

#include <cstddef>
#include <cstdint>

namespace emri {

constexpr int SCORE_THREADS = 512;   // one persistent workgroup of 8 waves per CU
constexpr int SCORE_WAVES = SCORE_THREADS / 64;
constexpr int SCORE_LDS_LEAD = 16;   // bytes ahead of each LDS half's first row
constexpr int STAGE_CHUNK_LOG2 = 10;
constexpr int STAGE_CHUNK = 1 << STAGE_CHUNK_LOG2;   // bytes one wave copies with one instruction (64 lanes x 16 B)

static_assert(SCORE_THREADS % 64 == 0, "whole waves only");
static_assert(SCORE_WAVES * 64 == SCORE_THREADS, "SCORE_WAVES counts the waves of a workgroup");
// The owner of the final chunk is taken as `last & (SCORE_WAVES - 1)` on the
// device and as `chunk % SCORE_WAVES` for the zero slots on the host; they
// agree only for a power-of-two wave count.
static_assert(SCORE_WAVES > 0 && (SCORE_WAVES & (SCORE_WAVES - 1)) == 0, "wave count must be a power of two");
static_assert(STAGE_CHUNK == 64 * 16, "a chunk is one 16-byte copy per lane");

// The wave that copies chunk c of a step.
constexpr int chunk_owner(int c) { return c & (SCORE_WAVES - 1); }

// Rows staged by the step that starts at row r0 (0 if r0 is past the end).
constexpr int step_rows(int n_seg, int r0, int G) { return r0 >= n_seg ? 0 : (n_seg - r0 < G ? n_seg - r0 : G); }

// Index of the final chunk of a block of `bytes` (> 0) bytes.
constexpr int last_chunk(int bytes) { return (bytes - 1) >> STAGE_CHUNK_LOG2; }

// Source byte offset, within the final chunk, of the lane whose own offset is
// lane_off: lanes past the block re-read its last 16 bytes.
constexpr int last_chunk_src(int bytes, int lane_off) {
  const int lim = bytes - 16 - last_chunk(bytes) * STAGE_CHUNK;
  return lane_off < lim ? lane_off : lim;
}

// Every copy that wave `wave` issues for a step of `bytes` (> 0) bytes, as
// f(chunk, src_off): the lane whose own offset is lane_off reads the block at
// byte src_off and writes LDS byte chunk * STAGE_CHUNK + lane_off of the
// half's rows.  The device pipeline and the host-side check both enumerate
// copies through this function.
template <class F>
constexpr void for_each_copy(int wave, int lane_off, int bytes, F &&f) {
  const int last = last_chunk(bytes);
  for (int c = wave; c < last; c += SCORE_WAVES) f(c, c * STAGE_CHUNK + lane_off);
  if (chunk_owner(last) == wave) f(last, last * STAGE_CHUNK + last_chunk_src(bytes, lane_off));
}

inline size_t stage_round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offset, from the start of a half's rows (after the lead-in), of zero
// slot j (may be negative: the slot below bin 0 of row 0 is in the lead-in).
constexpr int zero_slot_rel(int j, int pitch_bytes, int elem_bytes, int k_min, int k_max) {
  return (j >> 1) * pitch_bytes + elem_bytes * ((j & 1) ? k_max + 1 : k_min - 1);
}

struct Staging {
  int G, pitch_bytes, half_bytes;
  uint64_t slot_owner;        // byte j: wave that re-zeroes zero slot j after a copy (0xff: none)
  size_t lds;                 // bytes of dynamic LDS (both halves and a 16-byte tail)
};

// Staging geometry for one spectrogram and bin range.  G = rows_per_step if it
// is nonzero, else the most of 4, 2, 1 that fit; G > 1 needs a padding element
// after every row (row_pitch > n_bins), which holds the slot above k_max of a
// row and below bin 0 of the next.  Returns false if it does not fit.
inline bool make_staging(int n_bins, int row_pitch, int elem_bytes, int k_min, int k_max, int rows_per_step,
                         size_t lds_limit, Staging *out) {
  const int pitch_bytes = row_pitch * elem_bytes;
  auto half_of = [&](int G) { return (size_t)SCORE_LDS_LEAD + stage_round_up((size_t)G * pitch_bytes, STAGE_CHUNK); };
  auto fits = [&](int G) { return 2 * half_of(G) + SCORE_LDS_LEAD <= lds_limit; };
  const bool padded = row_pitch > n_bins;
  int G = 0;
  if (rows_per_step != 0) {
    if ((rows_per_step > 1 && !padded) || !fits(rows_per_step)) return false;
    G = rows_per_step;
  } else {
    for (int g : {4, 2, 1})
      if ((g == 1 || padded) && fits(g)) {
        G = g;
        break;
      }
    if (G == 0) return false;
  }
  const int half = (int)half_of(G);
  const int copied = half - SCORE_LDS_LEAD;     // bytes a full step writes
  uint64_t owner = ~0ull;
  for (int j = 0; j < 2 * G; ++j) {
    const int rel = zero_slot_rel(j, pitch_bytes, elem_bytes, k_min, k_max);
    const uint64_t w = (rel >= 0 && rel < copied) ? (uint64_t)chunk_owner(rel >> STAGE_CHUNK_LOG2) : 0xffull;
    owner = (owner & ~(0xffull << (8 * j))) | (w << (8 * j));
  }
  out->G = G;
  out->pitch_bytes = pitch_bytes;
  out->half_bytes = half;
  out->slot_owner = owner;
  out->lds = 2 * (size_t)half + SCORE_LDS_LEAD;
  return true;
}

}  // namespace emri
