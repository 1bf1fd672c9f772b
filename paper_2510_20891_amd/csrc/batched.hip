// C ABI of the batched form: plan many scoring problems into one persistent
// launch (work split by tiles of templates, weighted by segment count), then
// run it with kernels that only read device tables, so the run can be captured
// into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "score_internal.h"
#include "topk_internal.h"

using namespace emri;

namespace {

constexpr size_t kLdsLimit = 163840 - 256;   // LDS of a workgroup, less the static work-item slot
constexpr uint32_t kPlanMagic = 0x454d5242u;   // "EMRB"

// What score_batched_run needs, stored inside the caller's emri_batch_plan.
struct PlanData {
  uint32_t magic;
  int32_t n_problems;
  int32_t n_topk;
  int32_t cus;
  int64_t max_topk_n;
  BatchLaunch launch;
  const PrepJob *prep_jobs;
  const TopkJob *topk_jobs;
  const int32_t *topk_block_job;
  int64_t topk_blocks;
  int32_t n_items;
  int32_t has_work;
  int32_t topk_fast;           // some top-k job takes the sampled threshold
};
static_assert(sizeof(PlanData) <= sizeof(emri_batch_plan), "plan does not fit");

int elem_bytes(int dtype) { return dtype == EMRI_F16 ? 2 : 4; }

int check_problem(const emri_problem &pb, int i, int K, int dtype) {
  const emri_power &pw = pb.power;
  if (pw.dtype != EMRI_F32 && pw.dtype != EMRI_F16) return fail(EMRI_EINVAL, "problem %d: unknown power dtype", i);
  if (pw.dtype != dtype) return fail(EMRI_EINVAL, "problem %d: every problem must use the same power dtype", i);
  if (pw.n_seg < 0 || pw.n_bins < 1) return fail(EMRI_EINVAL, "problem %d: n_seg < 0 or n_bins < 1", i);
  if (pw.row_pitch < pw.n_bins || (pw.row_pitch % 8) != 0)
    return fail(EMRI_EINVAL, "problem %d: row_pitch must be a multiple of 8 and >= n_bins", i);
  if (!std::isfinite(pw.t_sft) || !(pw.t_sft > 0.0)) return fail(EMRI_EINVAL, "problem %d: bad t_sft", i);
  if ((int64_t)pw.row_pitch * elem_bytes(pw.dtype) > INT32_MAX) return fail(EMRI_ERANGE, "problem %d: row too long", i);
  if (pb.n_tmpl < 0 || pb.n_tmpl > INT32_MAX) return fail(EMRI_EINVAL, "problem %d: n_tmpl out of range", i);
  if (pb.top_k < 0 || pb.top_k > EMRI_MAX_TOPK) return fail(EMRI_EINVAL, "problem %d: top_k out of range", i);
  if (pb.reserved != 0) return fail(EMRI_EINVAL, "problem %d: reserved must be zero", i);
  const int k_max = pb.k_max < 0 ? pw.n_bins - 1 : pb.k_max;
  if (pb.k_min < 0 || k_max > pw.n_bins - 1 || pb.k_min > k_max)
    return fail(EMRI_EINVAL, "problem %d: bin range outside the row", i);
  if (pw.n_seg > 0 && !pw.data) return fail(EMRI_EINVAL, "problem %d: power data is NULL", i);
  if (pw.n_seg > 0 && !pb.f0) return fail(EMRI_EINVAL, "problem %d: f0 is NULL", i);
  if (pw.n_seg > 0 && K > 0 && !pb.U) return fail(EMRI_EINVAL, "problem %d: U is NULL", i);
  if (pb.n_tmpl > 0 && K > 0 && !pb.coeffs) return fail(EMRI_EINVAL, "problem %d: coeffs is NULL", i);
  if (pb.top_k > 0 && (!pb.topk_val || !pb.topk_idx)) return fail(EMRI_EINVAL, "problem %d: top-k outputs NULL", i);
  const void *ptrs[] = {pw.data, pb.f0, pb.U, pb.coeffs, pb.stat, pb.topk_val, pb.topk_idx};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(EMRI_EINVAL, "problem %d: device pointers must be 16-byte aligned", i);
  return EMRI_OK;
}

// Workspace layout of a batch.
struct Layout {
  size_t params, prep, topk_jobs, topk_blocks, items, counter, redo, seg, bound, stat, topk, total;
  std::vector<size_t> seg_off, bound_off, mtab_off, mseg_off, stat_off, topk_off;
};

int seg_stride_of(int K) { return (K + 2) & ~1; }

Layout make_layout(const emri_problem *pbs, int n, int K, int64_t max_items) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes > 0 ? bytes : 1, 256);
    return at;
  };
  L.params = take(sizeof(ScoreParams) * n);
  L.prep = take(sizeof(PrepJob) * n);
  L.topk_jobs = take(sizeof(TopkJob) * n);
  std::vector<int64_t> topk_n;
  for (int i = 0; i < n; ++i)
    if (pbs[i].top_k > 0) topk_n.push_back(pbs[i].n_tmpl);
  L.topk_blocks = take(sizeof(int32_t) * (size_t)topk_max_blocks(topk_n.data(), (int)topk_n.size()));
  L.items = take(sizeof(BatchItem) * (size_t)max_items);
  L.counter = take(2 * sizeof(int));
  L.redo = take(MIXED_REDO_BYTES);   // the mixed form's tile queue above K = 8
  L.seg = off;
  for (int i = 0; i < n; ++i) {
    const int ns = pbs[i].power.n_seg > 0 ? pbs[i].power.n_seg : 1;
    L.seg_off.push_back(take(sizeof(double) * ns * seg_stride_of(K)));
    L.bound_off.push_back(take(sizeof(double) * (EMRI_MAX_K + 1)));
    const size_t n4 = (size_t)((ns + 3) & ~3);
    L.mtab_off.push_back(take(n4 * mixed_row_bytes(MIXED_MAX_K)));
    L.mseg_off.push_back(take(n4 * sizeof(MixedSeg)));
    L.stat_off.push_back(pbs[i].stat ? 0 : take(sizeof(float) * pbs[i].n_tmpl));
    L.topk_off.push_back(pbs[i].top_k > 0 ? take(topk_workspace_bytes(pbs[i].top_k)) : 0);
  }
  L.total = off;
  return L;
}

int tile_of(int K, int tpl_choice) { return tpl_choice * SCORE_THREADS; }

int resolve_tpl(int K, int requested, int *tpl) {
  const int def = score_templates_per_lane(K, false), alt = score_templates_per_lane(K, true);
  if (requested == 0 || requested == def) {
    *tpl = def;
    return EMRI_OK;
  }
  if ((K == 8 || K == 16) && requested == alt) {
    *tpl = alt;
    return EMRI_OK;
  }
  return fail(EMRI_EUNSUPPORTED, "templates_per_lane %d is not compiled for K = %d", requested, K);
}

// Upper bound on the work items of a batch: one per tile of the smallest tile
// any option of this K compiles.
int64_t max_items_for(const emri_problem *pbs, int n, int K) {
  int tpl = score_templates_per_lane(K, false);
  if (K == 8 || K == 16) tpl = std::min(tpl, score_templates_per_lane(K, true));
  int64_t tile = (int64_t)tpl * SCORE_THREADS;
  if (K >= 1 && K <= MIXED_MAX_K) tile = std::min<int64_t>(tile, mixed_tile_templates(K));
  int64_t items = 0;
  for (int i = 0; i < n; ++i) items += (pbs[i].n_tmpl + tile - 1) / tile;
  return items > 0 ? items : 1;
}

}  // namespace

extern "C" int score_batched_tile_options(int32_t K, int32_t *out, int32_t *n_out) {
  clear_error();
  if (!out || !n_out) return fail(EMRI_EINVAL, "out or n_out is NULL");
  if (K < 0 || K > EMRI_MAX_K) return fail(EMRI_EINVAL, "K outside [0, %d]", EMRI_MAX_K);
  out[0] = score_templates_per_lane(K, false);
  *n_out = 1;
  if (K == 8 || K == 16) {
    out[1] = score_templates_per_lane(K, true);
    *n_out = 2;
  }
  return EMRI_OK;
}

static int batch_grid(int *grid) { return device_cu_count(grid); }

extern "C" int score_batched_workspace_size(const emri_problem *problems, int32_t n_problems, int32_t K,
                                            size_t *bytes) {
  clear_error();
  if (!bytes || (!problems && n_problems > 0)) return fail(EMRI_EINVAL, "NULL argument");
  if (n_problems < 0 || n_problems > (1 << 20)) return fail(EMRI_EINVAL, "n_problems out of range");
  if (K < 0 || K > EMRI_MAX_K) return fail(EMRI_EINVAL, "K outside [0, %d]", EMRI_MAX_K);
  const int dtype = n_problems > 0 ? problems[0].power.dtype : EMRI_F32;
  for (int i = 0; i < n_problems; ++i) {
    const int st = check_problem(problems[i], i, K, dtype);
    if (st) return st;
  }
  const Layout L = make_layout(problems, n_problems, K, max_items_for(problems, n_problems, K));
  *bytes = L.total;
  return EMRI_OK;
}

extern "C" int score_batched_plan(const emri_problem *problems, int32_t n_problems, int32_t K, const batch_opts *opts,
                                  void *workspace, size_t workspace_bytes, emri_batch_plan *plan, void *hip_stream) {
  clear_error();
  if (!plan || !workspace || (!problems && n_problems > 0)) return fail(EMRI_EINVAL, "NULL argument");
  if (n_problems < 0 || n_problems > (1 << 20)) return fail(EMRI_EINVAL, "n_problems out of range");
  if (K < 0 || K > EMRI_MAX_K) return fail(EMRI_EINVAL, "K outside [0, %d]", EMRI_MAX_K);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(EMRI_EINVAL, "workspace must be 256-byte aligned");
  batch_opts o{};
  if (opts) {
    o = *opts;
    for (int i = 0; i < 5; ++i)
      if (o.reserved[i] != 0) return fail(EMRI_EINVAL, "batch_opts.reserved must be zero");
  }
  if (o.precision != EMRI_PLAIN && o.precision != EMRI_MIXED)
    return fail(EMRI_EINVAL, "unknown precision %d", o.precision);
  const bool mixed = o.precision == EMRI_MIXED;
  if (mixed && (K < 1 || K > MIXED_MAX_K))
    return fail(EMRI_EUNSUPPORTED, "the mixed-precision form is built for 1 <= K <= %d, not %d", MIXED_MAX_K, K);
  if (mixed && o.rows_per_step != 0 && o.rows_per_step != 4)
    return fail(EMRI_EUNSUPPORTED, "the mixed-precision form stages 4 rows per step");
  if (mixed && o.templates_per_lane != 0 && o.templates_per_lane != mixed_templates_per_lane(K))
    return fail(EMRI_EUNSUPPORTED, "templates_per_lane %d is not compiled for the mixed form", o.templates_per_lane);
  if (o.rows_per_step != 0 && o.rows_per_step != 1 && o.rows_per_step != 2 && o.rows_per_step != 4)
    return fail(EMRI_EINVAL, "rows_per_step must be 0, 1, 2 or 4");
  const int dtype = n_problems > 0 ? problems[0].power.dtype : EMRI_F32;
  for (int i = 0; i < n_problems; ++i) {
    const int st = check_problem(problems[i], i, K, dtype);
    if (st) return st;
  }
  int tpl = 0, st = EMRI_OK;
  if (mixed)
    tpl = mixed_templates_per_lane(K);
  else if ((st = resolve_tpl(K, o.templates_per_lane, &tpl)) != EMRI_OK)
    return st;

  // staging geometry per problem (the requested rows per step, or the most
  // that fit); the launch takes the largest LDS footprint
  std::vector<Staging> stg(n_problems);
  size_t lds = 0;
  for (int i = 0; i < n_problems; ++i) {
    const emri_power &pw = problems[i].power;
    const int k_max = problems[i].k_max < 0 ? pw.n_bins - 1 : problems[i].k_max;
    const size_t mtab_lds = mixed ? round_up((size_t)((pw.n_seg + 3) & ~3) * mixed_row_bytes(K), 1024) : 0;
    if (!make_staging(pw.n_bins, pw.row_pitch, elem_bytes(pw.dtype), problems[i].k_min, k_max,
                      mixed ? 4 : o.rows_per_step, kLdsLimit - mtab_lds, &stg[i]))
      return fail(EMRI_EUNSUPPORTED, "problem %d: %d rows per step of %d bins do not fit in LDS", i,
                  mixed ? 4 : (o.rows_per_step ? o.rows_per_step : 1), pw.n_bins);
    lds = std::max(lds, mtab_lds + stg[i].lds);
  }
  int cus = 0;
  if ((st = batch_grid(&cus)) != EMRI_OK) return st;
  const Layout L = make_layout(problems, n_problems, K, max_items_for(problems, n_problems, K));
  if (workspace_bytes < L.total)
    return fail(EMRI_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, L.total);
  char *ws = reinterpret_cast<char *>(workspace);

  // per-problem tables
  std::vector<ScoreParams> params(n_problems);
  std::vector<PrepJob> preps(n_problems);
  std::vector<TopkJob> topks;
  int64_t max_topk_n = 0;
  bool any_fast = false;
  for (int i = 0; i < n_problems; ++i) {
    const emri_problem &pb = problems[i];
    const int k_max = pb.k_max < 0 ? pb.power.n_bins - 1 : pb.k_max;
    ScoreParams &p = params[i];
    std::memset(&p, 0, sizeof p);
    p.power = pb.power.data;
    p.seg = reinterpret_cast<const double *>(ws + L.seg_off[i]);
    p.bound = reinterpret_cast<const double *>(ws + L.bound_off[i]);
    p.coeffs = pb.coeffs;
    p.stat = pb.stat ? pb.stat : reinterpret_cast<float *>(ws + L.stat_off[i]);
    p.n_tmpl = pb.n_tmpl;
    p.n_seg = pb.power.n_seg;
    p.seg_stride = seg_stride_of(K);
    p.k_min = pb.k_min;
    p.k_max = k_max;
    p.pitch_bytes = stg[i].pitch_bytes;
    p.G = stg[i].G;
    p.half_bytes = stg[i].half_bytes;
    p.slot_owner = stg[i].slot_owner;
    p.one = 1.0f;
    if (mixed) {
      p.mtab = ws + L.mtab_off[i];
      p.mseg = ws + L.mseg_off[i];
      p.mtab_bytes = ((pb.power.n_seg + 3) & ~3) * mixed_row_bytes(K);
      if (K > 8) p.redo = reinterpret_cast<unsigned *>(ws + L.redo);
      p.redo_tag = (uint32_t)i;
    }
    PrepJob &pj = preps[i];
    std::memset(&pj, 0, sizeof pj);
    pj.f0 = pb.f0;
    pj.U = pb.U;
    pj.seg = reinterpret_cast<double *>(ws + L.seg_off[i]);
    pj.bound = reinterpret_cast<double *>(ws + L.bound_off[i]);
    pj.t_sft = pb.power.t_sft;
    pj.K = K;
    pj.n_seg = pb.power.n_seg;
    pj.seg_stride = seg_stride_of(K);
    if (mixed) {
      pj.mtab = ws + L.mtab_off[i];
      pj.mseg = ws + L.mseg_off[i];
      if (K > 8 && i == 0) pj.redo = reinterpret_cast<unsigned *>(ws + L.redo);   // clears the queue's count
    }
    if (pb.top_k > 0) {
      pj.topk = reinterpret_cast<TopkState *>(ws + L.topk_off[i]);
      topks.push_back(make_topk_job(p.stat, pb.n_tmpl, pb.top_k, pb.topk_val, pb.topk_idx, ws + L.topk_off[i]));
      topks.back().fast_r = topk_fast_rank(pb.n_tmpl, topks.back().kk);
      any_fast = any_fast || topks.back().fast_r != 0u;
      max_topk_n = std::max(max_topk_n, pb.n_tmpl);
    }
  }

  // work items: two tiles of one problem (a problem's odd last tile alone),
  // in decreasing order of cost (tiles x (segments + 4)), so the launch ends
  // on the cheapest items; workgroups claim them in this order
  const int64_t tile = mixed ? mixed_tile_templates(K) : tile_of(K, tpl);
  std::vector<BatchItem> items;
  std::vector<double> cost;
  for (int i = 0; i < n_problems; ++i) {
    const double w = (double)(((problems[i].power.n_seg + 3) & ~3) + 4);
    for (int64_t t = 0; t * tile < problems[i].n_tmpl; t += 2) {
      BatchItem it{};
      it.stream = i;
      it.begin = t * tile;
      it.end = std::min(problems[i].n_tmpl, (t + 2) * tile);
      items.push_back(it);
      cost.push_back(w * (double)((it.end - it.begin + tile - 1) / tile));
    }
  }
  std::vector<int> order(items.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  {
    std::vector<BatchItem> sorted(items.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = items[order[k]];
    items.swap(sorted);
  }
  if ((int64_t)items.size() > max_items_for(problems, n_problems, K) || items.size() > (size_t)INT32_MAX)
    return fail(EMRI_ERANGE, "work list longer than planned");
  const int grid = (int)std::min<size_t>((size_t)std::min(cus, 1024), std::max<size_t>(items.size(), 1));

  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t err = hipSuccess;
  auto copy = [&](size_t off, const void *src, size_t bytes) {
    if (bytes && err == hipSuccess) err = hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, stream);
  };
  copy(L.params, params.data(), sizeof(ScoreParams) * params.size());
  copy(L.prep, preps.data(), sizeof(PrepJob) * preps.size());
  const int64_t topk_blocks = topk_assign_blocks(topks.data(), (int)topks.size(), cus);
  std::vector<int32_t> block_job((size_t)topk_blocks);
  for (size_t j = 0; j < topks.size(); ++j)
    for (int b = 0; b < topks[j].nblk; ++b) block_job[(size_t)topks[j].first_block + b] = (int32_t)j;
  copy(L.topk_jobs, topks.data(), sizeof(TopkJob) * topks.size());
  copy(L.topk_blocks, block_job.data(), sizeof(int32_t) * block_job.size());
  copy(L.items, items.data(), sizeof(BatchItem) * items.size());
  // The tables are host vectors that go away when this call returns, and an
  // asynchronous copy from pageable memory may still be reading them: wait for
  // the copies (planning is a set-up step; score_batched_run never waits).
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "batched plan copies: %s", hipGetErrorString(err));

  PlanData pd{};
  pd.magic = kPlanMagic;
  pd.n_problems = n_problems;
  pd.n_topk = (int)topks.size();
  pd.cus = cus;
  pd.max_topk_n = max_topk_n;
  pd.launch.params = reinterpret_cast<const ScoreParams *>(ws + L.params);
  pd.launch.items = reinterpret_cast<const BatchItem *>(ws + L.items);
  pd.launch.counter = reinterpret_cast<int *>(ws + L.counter);
  pd.launch.n_items = (int)items.size();
  pd.launch.grid = grid;
  pd.launch.K = K;
  pd.launch.dtype = dtype;
  pd.launch.tpl = tpl;
  pd.launch.lds = lds;
  pd.launch.mixed = mixed ? 1 : 0;
  pd.launch.redo = (mixed && K > 8) ? reinterpret_cast<unsigned *>(ws + L.redo) : nullptr;
  pd.prep_jobs = reinterpret_cast<const PrepJob *>(ws + L.prep);
  pd.topk_jobs = reinterpret_cast<const TopkJob *>(ws + L.topk_jobs);
  pd.topk_block_job = reinterpret_cast<const int32_t *>(ws + L.topk_blocks);
  pd.topk_blocks = topk_blocks;
  pd.n_items = (int)items.size();
  pd.has_work = items.empty() ? 0 : 1;
  pd.topk_fast = any_fast ? 1 : 0;
  std::memset(plan, 0, sizeof *plan);
  std::memcpy(plan, &pd, sizeof pd);
  return EMRI_OK;
}

extern "C" int score_batched_run(const emri_batch_plan *plan, void *hip_stream) {
  clear_error();
  if (!plan) return fail(EMRI_EINVAL, "plan is NULL");
  PlanData pd;
  std::memcpy(&pd, plan, sizeof pd);
  if (pd.magic != kPlanMagic) return fail(EMRI_EINVAL, "plan was not made by score_batched_plan");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t err = launch_score_prep_batched(pd.prep_jobs, pd.n_problems, pd.launch.counter, stream);
  if (err == hipSuccess && pd.has_work)
    err = pd.launch.mixed ? launch_score_mixed_batched(pd.launch, stream) : launch_score_batched(pd.launch, stream);
  if (err == hipSuccess && pd.n_topk > 0) {
    TopkJobs J;
    std::memset(&J, 0, sizeof J);
    J.jobs = pd.topk_jobs;
    J.block_job = pd.topk_block_job;
    err = launch_topk_jobs(J, pd.topk_blocks, pd.max_topk_n, stream, 0, pd.topk_fast != 0);
  }
  if (err != hipSuccess) return fail(EMRI_EDEVICE, "batched launch: %s", hipGetErrorString(err));
  return EMRI_OK;
}
