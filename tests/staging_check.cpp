// Host-side check of the LDS row staging geometry used by the scoring kernels
// (paper_2510_20891_amd/csrc/staging_geom.h).  For many spectrogram shapes,
// bin ranges, element sizes, rows per step and segment counts it replays every
// copy of every staging step through the same for_each_copy / make_staging /
// zero_slot_rel functions the device code runs, on a simulated LDS, and checks:
//   * every global read lies inside the spectrogram, [0, n_seg * pitch_bytes);
//   * every LDS write lies inside the half being filled (after its lead-in);
//   * every zero slot a copy overwrites has an owner wave that re-zeroes it;
//   * after a step is published, every element a gather can reach (bins
//     k_min - 1 .. k_max + 1 of each staged row) holds that row's power or,
//     for the two slots, zero.
// Prints "ok <cases>" and exits 0, or prints the first failure and exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "staging_geom.h"

using namespace emri;

namespace {

constexpr long kZero = -1;       // LDS byte known to be zero
constexpr long kGarbage = -2;    // LDS byte never written

struct Case {
  int n_bins, row_pitch, elem, k_min, k_max, rows_per_step, n_seg;
  size_t lds_limit;
};

int g_fail = 0;

#define CHECK(cond, ...)                                                                                   \
  do {                                                                                                     \
    if (!(cond)) {                                                                                         \
      std::printf("FAIL n_bins=%d pitch=%d elem=%d k=[%d,%d] G=%d n_seg=%d lds=%zu: ", c.n_bins, c.row_pitch, \
                  c.elem, c.k_min, c.k_max, c.rows_per_step, c.n_seg, c.lds_limit);                         \
      std::printf(__VA_ARGS__);                                                                            \
      std::printf("\n");                                                                                   \
      g_fail = 1;                                                                                          \
      return false;                                                                                        \
    }                                                                                                      \
  } while (0)

bool run_case(const Case &c, bool *fitted) {
  Staging sg;
  *fitted = make_staging(c.n_bins, c.row_pitch, c.elem, c.k_min, c.k_max, c.rows_per_step, c.lds_limit, &sg);
  if (!*fitted) return true;
  const int G = sg.G;
  CHECK(sg.lds <= c.lds_limit, "LDS %zu over the limit", sg.lds);
  CHECK(sg.pitch_bytes == c.row_pitch * c.elem, "pitch bytes");
  CHECK(c.rows_per_step == 0 || G == c.rows_per_step, "G %d", G);
  const long hbm_bytes = (long)c.n_seg * sg.pitch_bytes;
  std::vector<long> lds(sg.lds, kGarbage);
  // init_lds: the lead-in of each half and the tail after the second half
  for (int t = 0; t < 3 * SCORE_LDS_LEAD; ++t) lds[(size_t)(t / SCORE_LDS_LEAD) * sg.half_bytes + t % SCORE_LDS_LEAD] = kZero;
  int half = 0;
  for (int r0 = 0; r0 < c.n_seg; r0 += G) {
    const int rows = step_rows(c.n_seg, r0, G);
    CHECK(rows >= 1 && rows <= G, "rows %d at r0 %d", rows, r0);
    const int bytes = rows * sg.pitch_bytes;
    const long half_start = (long)half * sg.half_bytes;
    const long rows_start = half_start + SCORE_LDS_LEAD;
    // which waves' copies write each zero slot of this step (waves run
    // concurrently: a slot may only be re-zeroed by the one wave that wrote it)
    long slot_at[8];
    int slot_writers[8];
    for (int j = 0; j < 2 * G; ++j) {
      slot_at[j] = rows_start + zero_slot_rel(j, sg.pitch_bytes, c.elem, c.k_min, c.k_max);
      slot_writers[j] = 0;
    }
    for (int wave = 0; wave < SCORE_WAVES; ++wave) {
      for (int lane = 0; lane < 64; ++lane) {
        const int lane_off = lane * 16;
        bool ok = true;
        for_each_copy(wave, lane_off, bytes, [&](int chunk, int src_off) {
          const long src = (long)r0 * sg.pitch_bytes + src_off;
          const long dst = rows_start + (long)chunk * STAGE_CHUNK + lane_off;
          if (src_off < 0 || src_off + 16 > bytes || src < 0 || src + 16 > hbm_bytes) {
            std::printf("read [%ld, %ld) outside the block or spectrogram (bytes %d, r0 %d)\n", src, src + 16, bytes, r0);
            ok = false;
          }
          if (dst < rows_start || dst + 16 > half_start + sg.half_bytes) {
            std::printf("write [%ld, %ld) outside half %d [%ld, %ld)\n", dst, dst + 16, half, rows_start,
                        half_start + (long)sg.half_bytes);
            ok = false;
          }
          for (int b = 0; b < 16 && ok; ++b) lds[dst + b] = src + b;
          for (int j = 0; j < 2 * G; ++j)
            if (slot_at[j] + c.elem > dst && slot_at[j] < dst + 16) slot_writers[j] |= 1 << wave;
        });
        CHECK(ok, "copy out of bounds (wave %d lane %d)", wave, lane);
      }
    }
    // pipe_publish: each wave, after its own copies, re-zeroes the slots it owns
    for (int j = 0; j < 2 * G; ++j) {
      const int rel = zero_slot_rel(j, sg.pitch_bytes, c.elem, c.k_min, c.k_max);
      const int owner = (int)((sg.slot_owner >> (8 * j)) & 0xffu);
      const long at = rows_start + rel;
      CHECK(at >= 0 && at + c.elem <= (long)sg.lds, "slot %d at %ld outside LDS", j, at);
      CHECK(slot_writers[j] == 0 || (owner != 0xff && slot_writers[j] == (1 << owner)),
            "slot %d written by waves 0x%x but owned by %d", j, slot_writers[j], owner);
      if (owner != 0xff) {
        CHECK(owner < SCORE_WAVES, "slot %d owner %d", j, owner);
        for (int b = 0; b < c.elem; ++b) lds[at + b] = kZero;
      }
    }
    // gathers: bins k_min - 1 .. k_max + 1 of each staged row
    for (int i = 0; i < rows; ++i) {
      for (int bin = c.k_min - 1; bin <= c.k_max + 1; ++bin) {
        const long at = rows_start + (long)i * sg.pitch_bytes + (long)c.elem * bin;
        CHECK(at >= 0 && at + c.elem <= (long)sg.lds, "gather of row %d bin %d at %ld outside LDS", r0 + i, bin, at);
        const bool slot = bin == c.k_min - 1 || bin == c.k_max + 1;
        for (int b = 0; b < c.elem; ++b) {
          const long want = slot ? kZero : (long)(r0 + i) * sg.pitch_bytes + (long)c.elem * bin + b;
          CHECK(lds[at + b] == want, "row %d bin %d byte %d holds %ld, want %ld (step r0 %d, half %d)", r0 + i, bin,
                b, lds[at + b], want, r0, half);
        }
      }
    }
    half ^= 1;
  }
  return true;
}

}  // namespace

int main() {
  const int elems[] = {2, 4};
  const int n_bins_list[] = {1, 2, 3, 7, 8, 9, 16, 31, 33, 128, 255, 256, 257, 511, 512, 513, 1023, 1025,
                             2049, 4321, 5001, 8193, 10241};
  const int gs[] = {0, 1, 2, 4};
  const int n_segs[] = {1, 2, 3, 4, 5, 7, 8, 9, 13, 30};
  long cases = 0, fitted = 0;
  for (int elem : elems)
    for (int n_bins : n_bins_list) {
      const int pitches[] = {(n_bins + 7) / 8 * 8, (n_bins + 8) / 8 * 8, (n_bins + 8) / 8 * 8 + 64};
      for (int pitch : pitches) {
        // whole row; interior range; a one-bin range; a range at the top edge
        const int ranges[4][2] = {{0, n_bins - 1},
                                  {n_bins > 4 ? 2 : 0, n_bins > 4 ? n_bins - 3 : n_bins - 1},
                                  {n_bins / 2, n_bins / 2},
                                  {n_bins - 1, n_bins - 1}};
        for (const auto &rg : ranges)
          for (int G : gs)
            for (int n_seg : n_segs)
              for (size_t lds_limit : {(size_t)163840, (size_t)163840 - 5 * 1024}) {
                const Case c{n_bins, pitch, elem, rg[0], rg[1], G, n_seg, lds_limit};
                bool fit = false;
                if (!run_case(c, &fit)) return 1;
                ++cases;
                fitted += fit;
              }
      }
    }
  if (g_fail) return 1;
  std::printf("ok %ld cases (%ld fit in LDS)\n", cases, fitted);
  return 0;
}
