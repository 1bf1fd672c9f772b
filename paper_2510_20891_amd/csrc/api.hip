// C ABI of score_tracks: argument validation, workspace layout and launches.
#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "score_internal.h"
#include "topk_internal.h"
#include "rescore_internal.h"

using namespace emri;

namespace {

constexpr size_t kLdsLimit = 163840;      // bytes of LDS a gfx950 workgroup may use

struct Layout {
  size_t seg_off, bound_off, mtab_off, mseg_off, redo_off, stat_off, topk_off, cand_val_off, cand_idx_off, total;
  int seg_stride;
};

int elem_bytes(int dtype) { return dtype == EMRI_F16 ? 2 : 4; }

int check_power(const emri_power *pw) {
  if (!pw) return fail(EMRI_EINVAL, "power is NULL");
  if (pw->dtype != EMRI_F32 && pw->dtype != EMRI_F16) return fail(EMRI_EINVAL, "unknown power dtype %d", pw->dtype);
  if (pw->n_seg < 0 || pw->n_bins < 1) return fail(EMRI_EINVAL, "n_seg must be >= 0 and n_bins >= 1");
  if (pw->row_pitch < pw->n_bins || (pw->row_pitch % 8) != 0)
    return fail(EMRI_EINVAL, "row_pitch %d must be a multiple of 8 and >= n_bins %d", pw->row_pitch, pw->n_bins);
  if (!std::isfinite(pw->t_sft) || !(pw->t_sft > 0.0)) return fail(EMRI_EINVAL, "t_sft must be finite and > 0");
  if ((int64_t)pw->row_pitch * elem_bytes(pw->dtype) > INT32_MAX) return fail(EMRI_ERANGE, "row too long");
  return EMRI_OK;
}

int make_layout(const emri_power *pw, int K, int64_t n_tmpl, int top_k, bool stat_in_ws, Layout *L) {
  L->seg_stride = (K + 2) & ~1;                  // f0T + K entries, even for 16-byte rows
  size_t off = 0;
  L->seg_off = off;
  off += round_up((size_t)(pw->n_seg > 0 ? pw->n_seg : 1) * L->seg_stride * sizeof(double), 256);
  L->bound_off = off;
  off += round_up((EMRI_MAX_K + 1) * sizeof(double), 256);
  // tables of the mixed-precision form (sized for its largest K)
  const size_t n4 = (size_t)((pw->n_seg + 3) & ~3);
  L->mtab_off = off;
  off += round_up((n4 > 0 ? n4 : 4) * mixed_row_bytes(MIXED_MAX_K), 256);
  L->mseg_off = off;
  off += round_up((n4 > 0 ? n4 : 4) * sizeof(MixedSeg), 256);
  L->redo_off = off;                             // tile queue of the reduced-chain launch
  off += round_up(MIXED_REDO_BYTES, 256);
  L->stat_off = off;
  if (stat_in_ws) off += round_up((size_t)n_tmpl * sizeof(float), 256);
  // the top-k state (sized for the candidates of a re-scoring mixed call,
  // which a plain call leaves unused) and the re-scored candidates
  const int n_cand = top_k > 0 ? rescore_candidates(top_k, n_tmpl) : 0;
  L->topk_off = off;
  off += topk_workspace_bytes(std::max(top_k, n_cand));
  L->cand_val_off = off;
  off += round_up((size_t)std::max(n_cand, 1) * sizeof(float), 256);
  L->cand_idx_off = off;
  off += round_up((size_t)std::max(n_cand, 1) * sizeof(int64_t), 256);
  L->total = off;
  return EMRI_OK;
}

int check_sizes(const emri_power *pw, int K, int64_t n_tmpl, int top_k) {
  int st = check_power(pw);
  if (st) return st;
  if (K < 0 || K > EMRI_MAX_K) return fail(EMRI_EINVAL, "K = %d outside [0, %d]", K, EMRI_MAX_K);
  if (n_tmpl < 0 || n_tmpl > INT32_MAX) return fail(EMRI_EINVAL, "n_tmpl = %lld outside [0, 2^31-1]", (long long)n_tmpl);
  if (top_k < 0 || top_k > EMRI_MAX_TOPK) return fail(EMRI_EINVAL, "top_k = %d outside [0, %d]", top_k, EMRI_MAX_TOPK);
  if ((int64_t)pw->n_seg * n_tmpl > (int64_t)1 << 62) return fail(EMRI_ERANGE, "n_tmpl * n_seg overflows");
  return EMRI_OK;
}

}  // namespace

extern "C" int score_tracks_workspace_size(const emri_power *power, int32_t K, int64_t n_tmpl, int32_t top_k,
                                           int32_t stat_in_workspace, size_t *bytes) {
  clear_error();
  if (!bytes) return fail(EMRI_EINVAL, "bytes is NULL");
  int st = check_sizes(power, K, n_tmpl, top_k);
  if (st) return st;
  Layout L;
  make_layout(power, K, n_tmpl, top_k, stat_in_workspace != 0, &L);
  *bytes = L.total;
  return EMRI_OK;
}

namespace {

// Scratch of score_tracks_noalloc: one copy per GPU, in the code object's
// device memory, held until the process ends.  Its address on a device comes
// from hipGetSymbolAddress with that device current (the array's name in host
// code is only a host-side stand-in).  Calls on one device share it.
constexpr size_t kNoallocScratchBytes = (size_t)4 << 20;
__device__ __attribute__((aligned(256))) unsigned char scratch[kNoallocScratchBytes];

int scratch_address(void **out) {
  static std::mutex mu;
  static void *addr[64] = {nullptr};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(EMRI_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !p)
      return fail(EMRI_EDEVICE, "static scratch of device %d: %s", dev, hipGetErrorString(err));
    addr[dev] = p;
  }
  *out = addr[dev];
  return EMRI_OK;
}

int score_tracks_impl(const emri_power *power, const double *f0, const double *U, int32_t K, const float *coeffs,
                      int64_t n_tmpl, int32_t top_k, float *stat, float *topk_val, int64_t *topk_idx, int32_t *bins,
                      int64_t *n_near_tie, const score_opts *opts, void *workspace, size_t workspace_bytes,
                      void *hip_stream, bool static_scratch, int n_harm = 0, const double *ratios = nullptr);

}  // namespace

extern "C" int score_tracks(const emri_power *power, const double *f0, const double *U, int32_t K,
                            const float *coeffs, int64_t n_tmpl, int32_t top_k, float *stat, float *topk_val,
                            int64_t *topk_idx, int32_t *bins, int64_t *n_near_tie, const score_opts *opts,
                            void *workspace, size_t workspace_bytes, void *hip_stream) {
  clear_error();
  return score_tracks_impl(power, f0, U, K, coeffs, n_tmpl, top_k, stat, topk_val, topk_idx, bins, n_near_tie, opts,
                           workspace, workspace_bytes, hip_stream, false);
}

extern "C" int score_tracks_noalloc(const emri_power *power, const double *f0, const double *U, int32_t K,
                                    const float *coeffs, int64_t n_tmpl, int32_t top_k, float *stat,
                                    float *topk_val, int64_t *topk_idx, int32_t *bins, int64_t *n_near_tie,
                                    const score_opts *opts, void *hip_stream) {
  clear_error();
  return score_tracks_impl(power, f0, U, K, coeffs, n_tmpl, top_k, stat, topk_val, topk_idx, bins, n_near_tie, opts,
                           nullptr, kNoallocScratchBytes, hip_stream, true);
}

extern "C" size_t score_tracks_noalloc_limit(void) { return kNoallocScratchBytes; }

extern "C" int score_tracks_harmonics(const emri_power *power, const double *f0, const double *U, int32_t K,
                                      const float *coeffs, int64_t n_tmpl, int32_t n_harm, const double *ratios,
                                      int32_t top_k, float *stat, float *topk_val, int64_t *topk_idx,
                                      const score_opts *opts, void *workspace, size_t workspace_bytes,
                                      void *hip_stream) {
  clear_error();
  if (n_harm < 1) return fail(EMRI_EINVAL, "n_harm must be >= 1");
  return score_tracks_impl(power, f0, U, K, coeffs, n_tmpl, top_k, stat, topk_val, topk_idx, nullptr, nullptr, opts,
                           workspace, workspace_bytes, hip_stream, false, n_harm, ratios);
}

namespace {

int score_tracks_impl(const emri_power *power, const double *f0, const double *U, int32_t K, const float *coeffs,
                      int64_t n_tmpl, int32_t top_k, float *stat, float *topk_val, int64_t *topk_idx, int32_t *bins,
                      int64_t *n_near_tie, const score_opts *opts, void *workspace, size_t workspace_bytes,
                      void *hip_stream, bool static_scratch, int n_harm, const double *ratios) {
  int st = check_sizes(power, K, n_tmpl, top_k);
  if (st) return st;
  int k_min = 0, k_max = power->n_bins - 1, precision = EMRI_PLAIN, rescore_top = 0;
  if (opts) {
    for (int i = 0; i < 4; ++i)
      if (opts->reserved[i] != 0) return fail(EMRI_EINVAL, "score_opts.reserved must be zero");
    k_min = opts->k_min;
    if (opts->k_max >= 0) k_max = opts->k_max;
    precision = opts->precision;
    rescore_top = opts->rescore_top;
  }
  if (rescore_top != 0 && rescore_top != 1) return fail(EMRI_EINVAL, "rescore_top must be 0 or 1");
  if (precision != EMRI_PLAIN && precision != EMRI_MIXED)
    return fail(EMRI_EINVAL, "unknown precision %d", precision);
  const bool mixed = precision == EMRI_MIXED;
  if (mixed && (K < 1 || K > MIXED_MAX_K))
    return fail(EMRI_EUNSUPPORTED, "the mixed-precision form is built for 1 <= K <= %d, not %d", MIXED_MAX_K, K);
  if (mixed && (bins || n_near_tie))
    return fail(EMRI_EUNSUPPORTED, "bins and n_near_tie come from the plain validation kernel only");
  const bool harm = n_harm > 0;
  if (harm) {
    if (!ratios) return fail(EMRI_EINVAL, "ratios is NULL");
    if (n_harm > HARMONICS_MAX_H) return fail(EMRI_EUNSUPPORTED, "at most %d harmonics, not %d", HARMONICS_MAX_H, n_harm);
    for (int h = 0; h < n_harm; ++h)
      if (!std::isfinite(ratios[h]) || !(ratios[h] > 0.0) || ratios[h] > 1024.0)
        return fail(EMRI_EINVAL, "harmonic ratio %d must be finite and in (0, 1024]", h);
    if (K < 1 || K > HARMONICS_MAX_K)
      return fail(EMRI_EUNSUPPORTED, "the multi-harmonic form is built for 1 <= K <= %d, not %d", HARMONICS_MAX_K, K);
    if (mixed) return fail(EMRI_EUNSUPPORTED, "the multi-harmonic form evaluates positions in FP64 only");
    if (bins || n_near_tie) return fail(EMRI_EUNSUPPORTED, "bins and n_near_tie are single-harmonic outputs");
  }
  if (k_min < 0 || k_max > power->n_bins - 1 || k_min > k_max)
    return fail(EMRI_EINVAL, "bin range [%d, %d] not inside [0, %d]", k_min, k_max, power->n_bins - 1);
  if (power->n_seg > 0 && !power->data) return fail(EMRI_EINVAL, "power->data is NULL");
  if (!f0 && power->n_seg > 0) return fail(EMRI_EINVAL, "f0 is NULL");
  if (!U && K > 0 && power->n_seg > 0) return fail(EMRI_EINVAL, "U is NULL");
  if (!coeffs && K > 0 && n_tmpl > 0) return fail(EMRI_EINVAL, "coeffs is NULL");
  if (top_k > 0 && (!topk_val || !topk_idx)) return fail(EMRI_EINVAL, "topk_val/topk_idx are NULL");
  if (!static_scratch && !workspace) return fail(EMRI_EINVAL, "workspace is NULL");
  const void *ptrs[] = {power->data, f0, U, coeffs, stat, topk_val, topk_idx, bins, n_near_tie};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(EMRI_EINVAL, "device pointers must be 16-byte aligned");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(EMRI_EINVAL, "workspace must be 256-byte aligned");
  Layout L;
  make_layout(power, K, n_tmpl, top_k, stat == nullptr, &L);
  if (static_scratch && L.total > workspace_bytes)
    return fail(EMRI_ENOMEM, "this call needs %zu bytes of scratch; the static scratch holds %zu (pass stat, or "
                "use score_tracks with a workspace)", L.total, workspace_bytes);
  if (workspace_bytes < L.total)
    return fail(EMRI_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, L.total);

  // LDS staging geometry: two halves of G consecutive rows (see score_internal.h)
  Staging sg;
  const int n4 = (power->n_seg + 3) & ~3;
  const int mtab_bytes = mixed ? n4 * mixed_row_bytes(K) : 0;
  const size_t mtab_lds = round_up((size_t)mtab_bytes, 1024);
  if (mixed) {
    // four rows per step (one round of matrix products) after the piece table
    if (!make_staging(power->n_bins, power->row_pitch, elem_bytes(power->dtype), k_min, k_max, 4,
                      kLdsLimit - mtab_lds, &sg))
      return fail(EMRI_EUNSUPPORTED,
                  "the mixed-precision form needs four padded rows of %d bins and the piece table in LDS",
                  power->n_bins);
  } else if (!make_staging(power->n_bins, power->row_pitch, elem_bytes(power->dtype), k_min, k_max, 0, kLdsLimit,
                           &sg)) {
    return fail(EMRI_EUNSUPPORTED, "a spectrogram row of %d bins does not fit twice in LDS", power->n_bins);
  }
  int cus = 0;
  if ((st = device_cu_count(&cus)) != EMRI_OK) return st;
  if (static_scratch && (st = scratch_address(&workspace)) != EMRI_OK) return st;

  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  char *ws = reinterpret_cast<char *>(workspace);
  double *seg = reinterpret_cast<double *>(ws + L.seg_off);
  double *bound = reinterpret_cast<double *>(ws + L.bound_off);
  float *stat_buf = stat ? stat : reinterpret_cast<float *>(ws + L.stat_off);
  const bool validate = bins != nullptr || n_near_tie != nullptr;

  hipError_t err = hipSuccess;
  if (power->n_seg > 0 || validate || top_k > 0) {
    PrepJob job{};
    job.f0 = f0;
    job.U = U;
    job.seg = seg;
    job.bound = bound;
    job.near_tie = reinterpret_cast<unsigned long long *>(n_near_tie);
    job.t_sft = power->t_sft;
    job.K = K;
    job.n_seg = power->n_seg;
    job.seg_stride = L.seg_stride;
    if (mixed) {
      job.mtab = ws + L.mtab_off;
      job.mseg = ws + L.mseg_off;
      if (K > 8) job.redo = reinterpret_cast<unsigned *>(ws + L.redo_off);
    }
    if (top_k > 0) job.topk = reinterpret_cast<TopkState *>(ws + L.topk_off);
    err = launch_score_prep(job, stream);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "score prep launch: %s", hipGetErrorString(err));
  }
  if (n_tmpl > 0) {
    ScoreParams p{};
    p.power = power->data;
    p.seg = seg;
    p.bound = bound;
    p.coeffs = coeffs;
    p.stat = stat_buf;
    p.bins = bins;
    p.near_tie = reinterpret_cast<unsigned long long *>(n_near_tie);
    p.n_tmpl = n_tmpl;
    p.n_seg = power->n_seg;
    p.seg_stride = L.seg_stride;
    p.k_min = k_min;
    p.k_max = k_max;
    p.pitch_bytes = sg.pitch_bytes;
    p.G = sg.G;
    p.half_bytes = sg.half_bytes;
    p.slot_owner = sg.slot_owner;
    p.one = 1.0f;
    if (mixed) {
      p.mtab = ws + L.mtab_off;
      p.mseg = ws + L.mseg_off;
      p.mtab_bytes = mtab_bytes;
      if (K > 8) p.redo = reinterpret_cast<unsigned *>(ws + L.redo_off);
    }
    // a plain launch with a top-k also runs the top-k's first key pass
    size_t lds = sg.lds;
    if (top_k > 0 && !mixed && !harm && !validate && power->n_seg > 0) {
      p.topk = reinterpret_cast<TopkState *>(ws + L.topk_off);
      p.topk_kk = (uint32_t)(n_tmpl < top_k ? n_tmpl : top_k);
      lds = std::max(lds, (size_t)TOPK_HIST * sizeof(uint32_t));
    }
    const int64_t units = (n_tmpl + SCORE_THREADS - 1) / SCORE_THREADS;
    const int grid = (int)(units < cus ? units : cus);
    p.per_block = (n_tmpl + grid - 1) / grid;
    if (harm && power->n_seg > 0) {
      p.topk = nullptr;
      err = launch_score_harmonics(p, K, power->dtype, n_harm, ratios, grid, sg.lds, stream);
    } else if (mixed && power->n_seg > 0) {
      err = launch_score_mixed(p, K, power->dtype, grid, mtab_lds + sg.lds, stream);
    } else if (power->n_seg == 0) {
      // no segment contributes: every statistic is zero; reuse the validation
      // kernel, whose segment loop is then empty
      err = launch_score(p, K, power->dtype, true, grid, sg.lds, stream);
    } else {
      err = launch_score(p, K, power->dtype, validate, grid, lds, stream);
    }
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "score launch: %s", hipGetErrorString(err));
  }
  if (top_k > 0 && mixed && rescore_top && n_tmpl > 0 && power->n_seg > 0) {
    // the leading candidates of the mixed statistic, re-scored with FP64
    // positions (the plain statistic), then ordered for the top-k
    const int n_cand = rescore_candidates(top_k, n_tmpl);
    float *cand_val = reinterpret_cast<float *>(ws + L.cand_val_off);
    int64_t *cand_idx = reinterpret_cast<int64_t *>(ws + L.cand_idx_off);
    err = launch_topk(stat_buf, n_tmpl, n_cand, cand_val, cand_idx, ws + L.topk_off, cus, stream, 0);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "top-k launch: %s", hipGetErrorString(err));
    RescoreParams r{};
    r.power = power->data;
    r.seg = seg;
    r.coeffs = coeffs;
    r.stat = stat_buf;
    r.cand_idx = cand_idx;
    r.cand_val = cand_val;
    r.n_tmpl = n_tmpl;
    r.n_cand = n_cand;
    r.n_seg = power->n_seg;
    r.seg_stride = L.seg_stride;
    r.K = K;
    r.row_pitch = power->row_pitch;
    r.k_min = k_min;
    r.k_max = k_max;
    err = launch_rescore(r, power->dtype, stream);
    if (err == hipSuccess) err = launch_rescore_select(cand_val, cand_idx, n_cand, top_k, topk_val, topk_idx, stream);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "re-scoring launch: %s", hipGetErrorString(err));
  } else if (top_k > 0) {
    const int first_pass = (n_tmpl > 0 && !mixed && !harm && !validate && power->n_seg > 0) ? 1 : 0;
    err = launch_topk(stat_buf, n_tmpl, top_k, topk_val, topk_idx, ws + L.topk_off, cus, stream, first_pass);
    if (err != hipSuccess) return fail(EMRI_EDEVICE, "top-k launch: %s", hipGetErrorString(err));
  }
  return EMRI_OK;
}

}  // namespace
