"""Benchmark: template-segment evaluations per second of the plain FP32 path on
the one-year stream (1e7 templates x 192 segments, K = 8, top-256), on one GPU.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one score_tracks call over the whole batch: track reconstruction,
nearest-bin gather, segment sum and top-k, with every input already resident
in HBM.  The spectrogram (build_sfts, GPU) and the basis (build_basis, host)
are built once before timing and reported separately.

Prints one JSON line.  `roofline` prices the scoring kernel against HBM
bandwidth on its algorithmic bytes, B = N_t (4K + 4) + N_t N_seg 4 +
N_seg N_bins 4 (every lookup counted once, no credit for on-chip reuse), per
launch; `cpu_baseline` times the FP64 oracle on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3       # MI355X published FP32 vector peak
FP64_VECTOR_PEAK_TFLOPS = 78.6        # MI355X published FP64 vector peak


def progress(msg: str) -> None:
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "score_fast_k8_f32_one_year_traffic.json")

_POOL_STATE = {}


def _pool_init(P, f0, U, C, t):
    _POOL_STATE.update(P=P, f0=f0, U=U, C=C, t=t)


def _oracle_chunk(bounds):
    import oracle
    s, e = bounds
    st = _POOL_STATE
    res = oracle.score_tracks(st["P"], st["f0"], st["U"], st["C"][s:e], st["t"], 0)
    return float(res["stat"].sum())


def cpu_baseline(P, f0, U, C, t_sft, n_sample: int) -> dict:
    """Oracle throughput on the first n_sample templates, one worker process per core."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    step = 16384
    chunks = [(s, min(s + step, n_sample)) for s in range(0, n_sample, step)]
    # fresh worker interpreters (no fork of a process that has loaded the GPU
    # runtime), each with one BLAS thread: the variables must be set before the
    # workers import numpy
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in saved:
        os.environ[v] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_pool_init, initargs=(P, f0, U, C[:n_sample], t_sft)) as pool:
        pool.map(_oracle_chunk, chunks[:cores])         # warm the workers
        t0 = time.perf_counter()
        pool.map(_oracle_chunk, chunks)
        wall = time.perf_counter() - t0
    for v, val in saved.items():
        if val is None:
            os.environ.pop(v, None)
        else:
            os.environ[v] = val
    evals = n_sample * P.shape[0]
    return {"value": evals / wall, "unit": "template-segment evals/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_sample} of the 1e7 templates x {P.shape[0]} segments, FP64 NumPy oracle, "
                      f"{cores} worker processes, {wall:.2f} s wall ({wall * cores:.0f} core-seconds)"}


def measured_traffic():
    """HBM bytes per launch of the scoring kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None if the kernel
    sources changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(PROFILE_TRAFFIC))
        h = hashlib.sha256()
        for src in rec["kernel_sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except (OSError, ValueError, KeyError):
        return None
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["kernel_sources_sha256"] else None


def copy_calibration(nbytes: int) -> int:
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters scale the kernel's."""
    import torch
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)
    return 0


# ----------------------------------------------------------------------------- forms
def _event_ms(fn, reps: int, stream=None) -> float:
    """Median wall time of fn() on the current stream, by HIP events, over reps runs."""
    import statistics
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return statistics.median(out)


def _event_ms_rotating(fns: dict, reps: int) -> dict:
    """Median wall time of each fn() by HIP events, the functions timed in
    rotation (one run of each per round, after one warm-up run each), so that
    every variant meets the same clock and power state of the chip."""
    import statistics
    import torch
    for fn in fns.values():
        fn()
    torch.cuda.synchronize()
    times = {name: [] for name in fns}
    for _ in range(reps):
        for name, fn in fns.items():
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times[name].append(e0.elapsed_time(e1))
    return {name: statistics.median(t) for name, t in times.items()}


def precision_form(st, reps: int = 7) -> dict:
    """Config 2: the one-year stream, 1e8 templates at K = 8 and K = 16, top-100.
    Plain FP32 (the plain path) vs plain FP16 vs mixed FP16; statistic error of
    the mixed form against the FP64 oracle on 2e5 sampled templates; top-100
    overlap against the oracle's exact top-100 (the oracle scores the union of
    the plain and mixed top-2000, which holds the true top-100 because the
    plain statistic is within 1e-5 of the oracle's).  mixed_f16_rescore is the
    mixed form with rescore_top: its top-100 candidates come from the mixed
    statistic and are re-scored with FP64 positions.  The error is also given
    over the sampled templates none of whose positions lies within 1e-3 bin of
    a half-integer (a moved bin needs such a position)."""
    import torch
    import oracle
    import paper_2510_20891_amd as emri
    dev = torch.device("cuda:0")
    n, top_k = 100_000_000, 100
    x_d = torch.from_numpy(st["x"]).to(dev)
    psd_d = torch.from_numpy(st["psd"]).to(dev)
    spec32 = emri.build_sfts(x_d, st["dt"], st["n_sft"], psd_d, dtype="f32")
    spec16 = emri.build_sfts(x_d, st["dt"], st["n_sft"], psd_d, dtype="f16")
    P16 = spec16.power().cpu().numpy().astype(np.float64)
    t_sft = spec16.t_sft
    res = {"workload": "one-year stream (192 x 8193), 1e8 templates uniform in the K-basis box, top-100",
           "power": "f16 for mixed and plain_f16, f32 for plain_f32"}
    ws = emri.Workspace()
    for K in (8, 16):
        f0, U, sv, lo, hi = emri.build_basis(st["tracks"], K)
        f0_d, U_d = torch.from_numpy(f0).to(dev), torch.from_numpy(U).to(dev)
        C_d = synth.device_coefficients(2, K, n, lo, hi, dev)
        out = {"stat": torch.empty(n, dtype=torch.float32, device=dev),
               "topk_val": torch.empty(top_k, dtype=torch.float32, device=dev),
               "topk_idx": torch.empty(top_k, dtype=torch.int64, device=dev)}
        variants = (("plain_f32", spec32, "plain", False), ("plain_f16", spec16, "plain", False),
                    ("mixed_f16", spec16, "mixed", False), ("mixed_f16_rescore", spec16, "mixed", True))
        call = lambda spec, prec, rs=False: emri.score_tracks(spec, f0_d, U_d, C_d, top_k, precision=prec,
                                                              rescore_top=rs, out=out, workspace=ws)
        times = _event_ms_rotating({name: (lambda spec=spec, prec=prec, rs=rs: call(spec, prec, rs))
                                    for name, spec, prec, rs in variants}, reps)
        runs = {name: {"ms": times[name], "evals_per_s": n * spec.n_seg / (times[name] * 1e-3)}
                for name, spec, prec, rs in variants}
        call(spec16, "mixed", True)
        resc_top = out["topk_idx"].cpu().numpy()
        resc_val = out["topk_val"].cpu().numpy()
        call(spec16, "plain")
        plain_idx = torch.topk(out["stat"], 2000).indices.cpu().numpy()
        call(spec16, "mixed")
        mixed_stat = out["stat"].clone()
        mixed_top = out["topk_idx"].cpu().numpy()
        # statistic error of the mixed form against the oracle (same FP16 power)
        rows = np.random.default_rng(20 + K).integers(0, n, 200_000)
        C_rows = C_d[torch.from_numpy(rows).to(dev)].cpu().numpy()
        o = oracle.score_tracks(P16, f0, U, C_rows, t_sft, 0)
        rel = np.abs(mixed_stat[torch.from_numpy(rows).to(dev)].cpu().numpy() - o["stat"]) / np.abs(o["stat"])
        x_rows = oracle.track_positions(f0, U, C_rows, t_sft)
        clear = ~(np.abs(x_rows - np.floor(x_rows) - 0.5) < 1e-3).any(axis=1)
        del x_rows
        # exact top-100 of the oracle over the candidate union
        mixed_cand = torch.topk(mixed_stat, 2000).indices.cpu().numpy()
        cand = np.unique(np.concatenate([plain_idx, mixed_cand]))
        oc = oracle.score_tracks(P16, f0, U, C_d[torch.from_numpy(cand).to(dev)].cpu().numpy(), t_sft, top_k)
        true_top = set(cand[oc["topk_idx"]].tolist())
        o_resc = oracle.score_tracks(P16, f0, U, C_d[torch.from_numpy(resc_top).to(dev)].cpu().numpy(), t_sft, 0)
        progress(f"precision form K={K}: mixed {runs['mixed_f16']['ms']:.2f} ms, plain f32 {runs['plain_f32']['ms']:.2f} ms")
        res[f"K{K}"] = {
            **{k: v for k, v in runs.items()},
            "speedup_mixed_vs_plain_f32": runs["plain_f32"]["ms"] / runs["mixed_f16"]["ms"],
            "speedup_mixed_vs_plain_f16": runs["plain_f16"]["ms"] / runs["mixed_f16"]["ms"],
            "speedup_mixed_rescore_vs_plain_f32": runs["plain_f32"]["ms"] / runs["mixed_f16_rescore"]["ms"],
            "stat_rel_err_vs_oracle": {"p50": float(np.quantile(rel, 0.5)), "p99": float(np.quantile(rel, 0.99)),
                                       "max": float(rel.max()), "sample": int(rows.size),
                                       "max_no_position_within_1e-3_of_half": float(rel[clear].max()),
                                       "templates_with_such_a_position": float(1.0 - clear.mean())},
            "top100_overlap": len(true_top & set(mixed_top.tolist())),
            "rescore_top100_overlap": len(true_top & set(resc_top.tolist())),
            "rescore_top100_max_rel_err_vs_oracle": float(np.max(np.abs(resc_val - o_resc["stat"]) / o_resc["stat"])),
        }
        del C_d, out, mixed_stat
        torch.cuda.empty_cache()
    return res


def batched_form(n_streams: int = 64, reps: int = 5) -> dict:
    """Config 3: 64 uneven streams (3-12 months, 48-192 segments, 1e5-1e7
    templates, top-256 each).  Stream by stream with score_tracks (plain FP32
    and FP16) vs one batched launch (tile shape from the autotuner) replayed
    from a captured HIP graph, plain and mixed, FP16 power."""
    import torch
    import paper_2510_20891_amd as emri
    from paper_2510_20891_amd import autotune
    dev = torch.device("cuda:0")
    K, top_k = 8, 256
    progress("batched form: generating streams")
    streams = synth.batched_streams(n_streams, cfg=3)
    progress("batched form: streams ready")
    probs16, probs32, evals, total = [], [], 0, 0
    for i, stv in enumerate(streams):
        f0, U, sv, lo, hi = emri.build_basis(stv["tracks"], K)
        x_d, psd_d = torch.from_numpy(stv["x"]).to(dev), torch.from_numpy(stv["psd"]).to(dev)
        s16 = emri.build_sfts(x_d, stv["dt"], stv["n_sft"], psd_d, dtype="f16")
        s32 = emri.build_sfts(x_d, stv["dt"], stv["n_sft"], psd_d, dtype="f32")
        C = synth.device_coefficients(3, i, stv["n_tmpl"], lo, hi, dev)
        f0_d, U_d = torch.from_numpy(f0).to(dev), torch.from_numpy(U).to(dev)
        probs16.append(emri.Problem(s16, f0_d, U_d, C, top_k=top_k))
        probs32.append(emri.Problem(s32, f0_d, U_d, C, top_k=top_k))
        evals += stv["n_tmpl"] * s16.n_seg
        total += stv["n_tmpl"]
    ws = emri.Workspace()

    def loop(probs, prec):
        for pb in probs:
            emri.score_tracks(pb.spec, pb.f0, pb.U, pb.coeffs, pb.top_k, precision=prec, workspace=ws)

    out = {"workload": f"{n_streams} streams, {total} templates, {evals:.4g} template-segment evaluations",
           "templates": total, "evals": evals}
    for name, probs, prec in (("per_stream_plain_f32", probs32, "plain"), ("per_stream_plain_f16", probs16, "plain")):
        ms = _event_ms(lambda: loop(probs, prec), reps)
        out[name] = {"ms": ms, "evals_per_s": evals / (ms * 1e-3)}
    progress(f"batched form: per-stream loops done")
    for prec in ("plain", "mixed"):
        plan, tune = autotune.tuned_plan(probs16, K, precision=prec, cache_path=None)
        progress(f"batched form: tuned {prec}: {tune.table}")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.run(side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run()
        ms = _event_ms(graph.replay, reps)
        # every stream's top-k is the standalone call's
        same = True
        for pb in probs16[:8]:
            ref = emri.score_tracks(pb.spec, pb.f0, pb.U, pb.coeffs, pb.top_k, precision=prec)
            torch.cuda.synchronize()
            same &= bool(torch.equal(ref["topk_idx"], pb.topk_idx) and torch.equal(ref["stat"], pb.stat))
        out[f"batched_{prec}_f16_graph"] = {
            "ms": ms, "evals_per_s": evals / (ms * 1e-3), "tile": {"rows_per_step": tune.rows_per_step,
                                                                    "templates_per_lane": tune.templates_per_lane},
            "autotune_table_ms": tune.table, "equals_standalone_first8": same}
        del graph
    base = out["per_stream_plain_f32"]["ms"]
    out["speedup_batched_plain_vs_per_stream_f32"] = base / out["batched_plain_f16_graph"]["ms"]
    out["speedup_batched_mixed_vs_per_stream_f32"] = base / out["batched_mixed_f16_graph"]["ms"]
    del probs16, probs32
    torch.cuda.empty_cache()
    return out


def serving_form(seconds: float = 32.0, warmup: float = 2.0, precision: str = "plain",
                 sweep_rates=(8000.0, 32000.0, 128000.0), sweep_seconds: float = 6.0) -> dict:
    """Config 4: 16 resident one-year FP16 spectrograms with a shared K = 8 basis;
    Poisson arrivals at 2000 requests/s of floor(logU[256, 65536]) templates
    against a uniform random stream, top-32 each; latency over the arrivals
    after the first ``warmup`` seconds.  Then a load sweep: the same server at
    higher arrival rates for ``sweep_seconds`` each (first second excluded),
    where requests overlap and batches grow, up to the device's throughput."""
    import torch
    import paper_2510_20891_amd as emri
    from paper_2510_20891_amd.serving import GpuExecutor, Request, Server
    dev = torch.device("cuda:0")
    K, n_streams = 8, 16
    specs, f0s, Us, segs = [], [], [], []
    basis = None
    for s in range(n_streams):
        stv = synth.stream_config1(stream=s, cfg=4)
        if basis is None:
            basis = emri.build_basis(stv["tracks"], K)
        x_d, psd_d = torch.from_numpy(stv["x"]).to(dev), torch.from_numpy(stv["psd"]).to(dev)
        specs.append(emri.build_sfts(x_d, stv["dt"], stv["n_sft"], psd_d, dtype="f16"))
        segs.append(specs[-1].n_seg)
    f0, U, sv, lo, hi = basis
    f0_d, U_d = torch.from_numpy(f0).to(dev), torch.from_numpy(U).to(dev)
    pool = synth.coefficients(4, 0, 1 << 22, lo, hi)
    reqs = [Request(r["rid"], r["stream"], pool[r["offset"]:r["offset"] + r["n"]], r["top_k"], r["t"])
            for r in synth.serving_requests(n_streams, 2000.0, seconds, cfg=4, pool_size=pool.shape[0])]
    slots, max_t, max_r = 3, 1 << 21, 512
    ex = GpuExecutor(specs, [f0_d] * n_streams, [U_d] * n_streams, K, slots, max_t, max_r, 32, precision)
    budget = 2 << 30
    srv = Server(ex, K, hbm_budget=budget, max_batch_templates=max_t, max_requests=max_r, slots=slots,
                 seg_counts=segs)
    # warm the kernels and the plan path
    warm = [Request(-1, 0, pool[:1024], 32, 0.0)]
    Server(ex, K, budget, max_t, max_r, slots).run(warm)
    progress(f"serving form: {len(reqs)} requests over {seconds:g} s")
    srv.run(reqs)
    st = srv.stats(reqs, warmup_s=warmup)
    progress(f"serving form: p50 {st.latency_ms['p50']:.2f} ms, p99 {st.latency_ms['p99']:.2f} ms")
    # a sample of results against standalone calls
    g = np.random.default_rng(5)
    same = True
    for r in [reqs[i] for i in g.integers(0, len(reqs), 24)]:
        ref = emri.score_tracks(specs[r.stream], f0_d, U_d, torch.from_numpy(r.coeffs).to(dev), 32, precision=precision)
        torch.cuda.synchronize()
        same &= bool(np.array_equal(ref["topk_idx"].cpu().numpy(), r.topk_idx)
                     and np.array_equal(ref["topk_val"].cpu().numpy(), r.topk_val))
    sweep = []
    for rate in sweep_rates:
        rq = [Request(r["rid"], r["stream"], pool[r["offset"]:r["offset"] + r["n"]], r["top_k"], r["t"])
              for r in synth.serving_requests(n_streams, rate, sweep_seconds, cfg=40 + int(rate) % 97,
                                              pool_size=pool.shape[0])]
        sv = Server(ex, K, hbm_budget=budget, max_batch_templates=max_t, max_requests=max_r, slots=slots,
                    seg_counts=segs)
        sv.run(rq)
        ss = sv.stats(rq, warmup_s=1.0)
        sweep.append({"offered_req_per_s": rate, "requests": ss.n_requests, "latency_ms": ss.latency_ms,
                      "throughput_req_per_s": ss.n_requests / ss.wall_s,
                      "throughput_evals_per_s": ss.evals / ss.wall_s, "batches": ss.batches,
                      "mean_batch_requests": ss.mean_batch_requests, "max_queue": ss.max_queue})
        progress(f"serving sweep {rate:g} req/s: p50 {ss.latency_ms['p50']:.2f} ms, p99 {ss.latency_ms['p99']:.2f} ms, "
                 f"{ss.mean_batch_requests:.1f} requests per batch")
    return {"workload": f"16 resident one-year FP16 spectrograms, Poisson 2000 req/s for {seconds:g} s "
                        f"(first {warmup:g} s excluded), logU[256, 65536] templates, top-32, precision {precision}",
            "requests": st.n_requests, "latency_ms": st.latency_ms,
            "throughput_evals_per_s": st.evals / st.wall_s, "throughput_req_per_s": st.n_requests / st.wall_s,
            "batches": st.batches, "mean_batch_requests": st.mean_batch_requests, "max_queue": st.max_queue,
            "slots": slots, "hbm_budget_bytes": budget, "same_as_standalone_24_sampled": same,
            "load_sweep": sweep}


def harmonics_form(st, n: int = 10_000_000, reps: int = 5) -> dict:
    """The multi-harmonic statistic (Sec. IV) on the one-year workload: 1e7
    templates, K = 8, top-256, FP32 power, harmonics at ratios 1, 1/2, 3/2 of
    the searched track (the m = 2, 1, 3 harmonics of a circular orbit), beside
    the single-harmonic call on the same batch.

    Roofline: the harmonics' power lookups are LDS gathers from rows already
    staged for the searched harmonic, so counted as HBM bytes they exceed the
    HBM peak (reported as lookup_GBps); the form is priced instead on its FP64
    arithmetic, 2 (K + H) flops per template and segment (K fused
    multiply-adds for the position, one per harmonic that scales and rounds),
    against the FP64 vector peak."""
    import torch
    import paper_2510_20891_amd as emri
    dev = torch.device("cuda:0")
    K, top_k, ratios = 8, 256, (1.0, 0.5, 1.5)
    f0, U, sv, lo, hi = emri.build_basis(st["tracks"], K)
    f0_d, U_d = torch.from_numpy(f0).to(dev), torch.from_numpy(U).to(dev)
    C_d = torch.from_numpy(synth.coefficients(1, 0, n, lo, hi)).to(dev)
    spec = emri.build_sfts(torch.from_numpy(st["x"]).to(dev), st["dt"], st["n_sft"],
                           torch.from_numpy(st["psd"]).to(dev))
    ws = emri.Workspace()
    out = {"stat": torch.empty(n, dtype=torch.float32, device=dev),
           "topk_val": torch.empty(top_k, dtype=torch.float32, device=dev),
           "topk_idx": torch.empty(top_k, dtype=torch.int64, device=dev)}
    ms_h = _event_ms(lambda: emri.score_tracks_harmonics(spec, f0_d, U_d, C_d, ratios, top_k, out=out,
                                                        workspace=ws), reps)
    ms_h0 = _event_ms(lambda: emri.score_tracks_harmonics(spec, f0_d, U_d, C_d, ratios, 0, out=out,
                                                         workspace=ws), reps)
    ms_1 = _event_ms(lambda: emri.score_tracks(spec, f0_d, U_d, C_d, top_k, out=out, workspace=ws), reps)
    H, n_seg = len(ratios), spec.n_seg
    b_look = n * (4 * K + 4) + n * n_seg * H * 4 + n_seg * spec.n_bins * 4
    flops = 2 * (K + H) * n * n_seg
    achieved = flops / (ms_h0 * 1e-3) / 1e12
    progress(f"harmonics form: {ms_h:.2f} ms for {H} harmonics, {ms_1:.2f} ms for one")
    return {"workload": f"one-year stream, {n} templates x {n_seg} segments, K = {K}, harmonics {list(ratios)}, "
                        f"top-{top_k}, FP32 power, FP64 positions",
            "ms": ms_h, "kernel_ms": ms_h0, "single_harmonic_ms": ms_1,
            "evals_per_s": n * n_seg / (ms_h * 1e-3),
            "harmonic_evals_per_s": n * n_seg * H / (ms_h * 1e-3),
            "cost_vs_single": ms_h / ms_1,
            "lookup_GBps": b_look / (ms_h0 * 1e-3) / 1e9,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "algorithmic_flops_per_eval": 2 * (K + H),
                         "algorithmic_flops_per_launch": flops}}


CHIRP_M = 256                       # template FFT length of the chirp kernel


def chirp_flops_per_eval(p_half: int = 100) -> int:
    """Algorithmic FP32 flops of one (template, segment) linear-chirp
    evaluation: the template's M-point FFT at 5 M log2 M, its M windowed
    samples at 6 flops each (sine and cosine not counted), and 14 flops per
    window bin (PSD weighting, the complex inner product and |H|^2)."""
    return 5 * CHIRP_M * 8 + 6 * CHIRP_M + 14 * (2 * p_half + 1)


def chirp_evaluated_segments(f0, U, C, t_sft: float, n_bins: int, f_min: float = 10.0 ** -3.5,
                             fdot_min: float = 1e-13, chunk: int = 100_000) -> int:
    """Template-segment pairs the linear-chirp statistic evaluates (host,
    FP64): those that pass the fddot limit and the cut-offs and whose central
    bin rint(f T) lies in the row.  Finite differences as the library takes
    them: central inside, second-order one-sided fdot at the ends, the
    neighbour's fddot at the ends (at least three segments)."""
    T = float(t_sft)
    total = 0
    for i in range(0, C.shape[0], chunk):
        f = f0[None, :] + C[i:i + chunk].astype(np.float64) @ U.T
        fd = np.empty_like(f)
        fd[:, 1:-1] = (f[:, 2:] - f[:, :-2]) / (2.0 * T)
        fd[:, 0] = (-3.0 * f[:, 0] + 4.0 * f[:, 1] - f[:, 2]) / (2.0 * T)
        fd[:, -1] = (3.0 * f[:, -1] - 4.0 * f[:, -2] + f[:, -3]) / (2.0 * T)
        fdd = np.empty_like(f)
        fdd[:, 1:-1] = (f[:, 2:] - 2.0 * f[:, 1:-1] + f[:, :-2]) / (T * T)
        fdd[:, 0], fdd[:, -1] = fdd[:, 1], fdd[:, -2]
        k0 = np.rint(f * T)
        use = (np.abs(fdd) * T ** 3 / 6.0 <= 1.0) & (f >= f_min) & (fd >= fdot_min) & (k0 >= 0) & (k0 < n_bins)
        total += int(use.sum())
    return total


def chirp_form(st, n: int = 1_000_000, reps: int = 3) -> dict:
    """The linear-chirp statistic (Sec. II B) on the one-year stream's
    whitened complex SFTs: 1e6 templates, K = 8, 2P + 1 = 201 bins, cut-offs
    of Sec. II D, top-256.  Arithmetic-bound: the roofline counts
    chirp_flops_per_eval flops per template and segment against the FP32
    vector peak, for the template-segment pairs it evaluates (those that
    pass the cuts, counted on the host)."""
    import torch
    import paper_2510_20891_amd as emri
    dev = torch.device("cuda:0")
    K, top_k = 8, 256
    f0, U, sv, lo, hi = emri.build_basis(st["tracks"], K)
    f0_d, U_d = torch.from_numpy(f0).to(dev), torch.from_numpy(U).to(dev)
    C = synth.coefficients(1, 0, n, lo, hi)
    C_d = torch.from_numpy(C).to(dev)
    psd_d = torch.from_numpy(st["psd"]).to(dev)
    spec = emri.build_sfts(torch.from_numpy(st["x"]).to(dev), st["dt"], st["n_sft"], psd_d, dtype="c32")
    ws = emri.Workspace()
    out = {"stat": torch.empty(n, dtype=torch.float32, device=dev),
           "topk_val": torch.empty(top_k, dtype=torch.float32, device=dev),
           "topk_idx": torch.empty(top_k, dtype=torch.int64, device=dev)}
    ms = _event_ms(lambda: emri.score_tracks_chirp(spec, psd_d, f0_d, U_d, C_d, top_k, out=out, workspace=ws), reps)
    ms0 = _event_ms(lambda: emri.score_tracks_chirp(spec, psd_d, f0_d, U_d, C_d, 0, out=out, workspace=ws), reps)
    n_seg = spec.n_seg
    evaluated = chirp_evaluated_segments(f0, U, C, spec.t_sft, spec.n_bins)
    flops = chirp_flops_per_eval() * evaluated
    achieved = flops / (ms0 * 1e-3) / 1e12
    progress(f"chirp form: {ms:.1f} ms for {n} templates ({achieved:.1f} TFLOP/s)")
    return {"workload": f"one-year stream's complex SFTs ({n_seg} x {spec.n_bins}), {n} templates, K = {K}, "
                        f"201-bin linear-chirp statistic, f >= 10^-3.5 Hz, fdot >= 1e-13 Hz/s, top-{top_k}",
            "ms": ms, "kernel_ms": ms0,
            "evals_per_s": n * n_seg / (ms * 1e-3),
            "evaluated_segments": evaluated,
            "evaluated_fraction": evaluated / (n * n_seg),
            "evaluated_evals_per_s": evaluated / (ms * 1e-3),
            "templates_per_s": n / (ms * 1e-3),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                         "algorithmic_flops_per_eval": chirp_flops_per_eval(),
                         "algorithmic_flops_per_launch": flops},
            "paper_context": "about 1.1 h for ~1e7 evaluations of the 201-bin statistic in the search of Sec. II D "
                             "on one unnamed GPU"}


def search_form(n_gen: int = 525, n_walk: int = 512, n_draw: int = 1024, n_chunks: int = 48,
                n_noise: int = 8, reps: int = 3) -> dict:
    """The population search of Sec. II D over progressive durations, on a
    one-year stream whose harmonic plunges at 0.7 of the data (192 segments,
    K = 8 basis of tracks that plunge at the end of the data): 48 chains on
    the first 19..192 segments (the basis shifted to end each track at the
    end of its data), 1024 seed candidates and 512 walkers each, 525
    differential-evolution generations captured into one HIP graph (all chains
    advance together, a pair of generations per launch pair, each launch
    forming, scoring and selecting); FP32 power, FP64 positions.  Each
    duration's best statistic is normalised by its mean and standard
    deviation over the same search on n_noise noise-only streams; the best
    normalised duration should sit at the injected plunge.  The same search
    is also run with the injection at SNR 60 (same noise, same normalisation)."""
    import torch
    import paper_2510_20891_amd as emri
    from paper_2510_20891_amd import search as drv
    dev = torch.device("cuda:0")
    K = 8
    st = synth.stream_progressive(stream=0)
    f0, U, sv, lo, hi = emri.build_basis(st["tracks"], K)
    f0_d, U_d = torch.from_numpy(f0).to(dev), torch.from_numpy(U).to(dev)
    lo_d, hi_d = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)

    def one_search(stv, seed, timed=False):
        x_d, psd_d = torch.from_numpy(stv["x"]).to(dev), torch.from_numpy(stv["psd"]).to(dev)
        spec = emri.build_sfts(x_d, stv["dt"], stv["n_sft"], psd_d)
        durations = drv.progressive_durations(spec.n_seg, n_chunks)
        chains = [drv.shifted_chain(spec, f0_d, U_d, lo_d, hi_d, n, n_walk) for n in durations]
        dr = [synth.search_seed_draws(seed, c, n_draw, lo, hi) for c in range(len(chains))]
        draws = torch.from_numpy(np.concatenate([d[0] for d in dr])).to(dev)
        finit = torch.from_numpy(np.concatenate([d[1] for d in dr])).to(dev)
        r1, r2, F = synth.device_generation_draws(seed, n_gen, [c.n_walkers for c in chains], dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run = drv.prepare(chains, K, draws, finit, r1, r2, F)
        torch.cuda.synchronize()
        out = {"durations": durations, "setup_s": time.perf_counter() - t0, "spec": spec, "chains": chains}
        if timed:
            out["replay_ms"] = _event_ms(run.graph.replay, reps)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            emri.search_seed(chains, K, draws, finit)
            ev1.record()
            torch.cuda.synchronize()
            out["seed_ms"] = ev0.elapsed_time(ev1)
        else:
            emri.search_seed(chains, K, draws, finit)
        run.graph.replay()                     # the reported search: seeded, then n_gen generations
        out["best"] = run.plan.best()["stat"].cpu().numpy()
        return out, run

    progress("search form: signal stream")
    sig, run = one_search(st, 7, timed=True)
    progress(f"search form: {sig['replay_ms'] / n_gen * 1e3:.1f} us per generation")
    bests = []
    for r in range(n_noise):
        stn = synth.stream_progressive(stream=100 + r, snr=None)
        o, _ = one_search(stn, 8 + r)
        bests.append(o["best"])
        progress(f"search form: noise-only search {r + 1}/{n_noise}")
    mean, sd = emri.search_noise_moments(torch.from_numpy(np.stack(bests).astype(np.float32)).to(dev))
    normed = run.plan.best(mean, sd)["norm"].cpu().numpy()
    durations = sig["durations"]
    # the same search on the same stream recipe with a louder injection (SNR 60)
    st60 = synth.stream_progressive(stream=0, snr=60.0)
    loud, run60 = one_search(st60, 7)
    normed60 = run60.plan.best(mean, sd)["norm"].cpu().numpy()
    progress("search form: SNR-60 search done")
    walkers = n_walk * len(durations)
    evals_gen = n_walk * sum(durations)
    # the injected track on the duration that ends at its plunge, projected on
    # that chain's basis rows and scored: what the search should reach there
    inj = st["injection"]
    n_true = int(round(inj["t_plunge"] / (st["n_sft"] * st["dt"])))
    c = int(np.argmin([abs(n - n_true) for n in durations]))
    n_c = durations[c]
    f_true = synth.chirp_frequency(st["t_mid"][:n_c], inj["f0"], inj["tau"])
    f0_c, U_c = f0[len(f0) - n_c:], U[len(f0) - n_c:]
    c_true = np.linalg.lstsq(U_c, f_true - f0_c, rcond=None)[0].astype(np.float32)[None, :]
    ch = sig["chains"][c]
    s_true = emri.score_tracks(ch.spec, ch.f0, ch.U, torch.from_numpy(c_true).to(dev), 1)["stat"]
    torch.cuda.synchronize()
    j = int(np.argmax(normed))
    j60 = int(np.argmax(normed60))
    inj60 = st60["injection"]
    n_true60 = int(round(inj60["t_plunge"] / (st60["n_sft"] * st60["dt"])))
    return {
        "workload": f"progressive search of a one-year stream whose harmonic plunges at 0.7 of the data: "
                    f"{len(durations)} durations ({durations[0]}..{durations[-1]} segments, basis shifted to end each "
                    f"track at the data's end), {n_draw} seed candidates and {n_walk} walkers per duration, {n_gen} DE "
                    f"generations in one HIP graph, K = {K}, FP32 power, FP64 positions; noise normalisation from "
                    f"{n_noise} noise-only streams",
        "walkers_per_generation": walkers,
        "evals_per_generation": evals_gen,
        "ms_per_generation": sig["replay_ms"] / n_gen,
        "template_segment_evals_per_s": evals_gen * n_gen / (sig["replay_ms"] * 1e-3),
        "statistic_evaluations_per_search": walkers * n_gen + n_draw * len(durations),
        "search_ms": sig["replay_ms"] + sig["seed_ms"],
        "seed_ms": sig["seed_ms"],
        "plan_and_capture_s": sig["setup_s"],
        "injected_plunge_segments": n_true,
        "best_normalised": float(normed[j]), "best_duration_segments": int(durations[j]),
        "normalised_by_duration": [round(float(v), 3) for v in normed],
        "found_stat_at_plunge_duration": float(sig["best"][c]),
        "injection_stat_at_plunge_duration": float(s_true[0]),
        "snr60": {"injected_plunge_segments": n_true60, "best_normalised": float(normed60[j60]),
                  "best_duration_segments": int(durations[j60]),
                  "found_stat_at_plunge_duration": float(loud["best"][c])},
        "paper_context": "about 1.1 h for ~1e7 statistic evaluations on one unnamed GPU (201-bin linear-chirp "
                         "statistic with Adam + DE, 48 durations x 512 walkers x 525 iterations)",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--templates", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=1 << 22)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="precision,batched,serving,search,harmonics,chirp",
                    help="comma-separated forms measured after the headline "
                         "(precision, batched, serving, search, harmonics, chirp, or none)")
    ap.add_argument("--serve-seconds", type=float, default=32.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (reference for traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(templates would shard across GPUs, each keeping its local top-k, merged by one exchange)",
              file=sys.stderr)
        return 2

    # ---- inputs (host), before any GPU initialisation -------------------------------
    progress("generating the one-year stream")
    st = synth.stream_config1(stream=0)
    n = args.templates
    K, top_k = st["K"], st["top_k"]

    import paper_2510_20891_amd as emri
    emri.load()
    t0 = time.perf_counter()
    f0, U, sv, lo, hi = emri.build_basis(st["tracks"], K)
    t_basis = time.perf_counter() - t0
    C = synth.coefficients(1, 0, n, lo, hi)

    cpu = None
    if not args.no_cpu:
        import oracle
        P_host = oracle.build_sfts(st["x"], st["dt"], st["n_sft"], st["psd"])
        progress("timing the oracle on the host")
        cpu = cpu_baseline(P_host, f0, U, C, st["n_sft"] * st["dt"], min(args.cpu_sample, n))
        progress(f"oracle: {cpu['value']:.3g} evals/s on {cpu['cores']} cores")

    # ---- GPU -------------------------------------------------------------------------
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x_d = torch.from_numpy(st["x"]).to(dev)
    psd_d = torch.from_numpy(st["psd"]).to(dev)
    f0_d = torch.from_numpy(f0).to(dev)
    U_d = torch.from_numpy(U).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C_d = torch.from_numpy(C).to(dev)
    torch.cuda.synchronize()
    t_h2d = time.perf_counter() - t0

    spec = emri.build_sfts(x_d, st["dt"], st["n_sft"], psd_d)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        spec = emri.build_sfts(x_d, st["dt"], st["n_sft"], psd_d)
    ev1.record()
    torch.cuda.synchronize()
    t_sfts_ms = ev0.elapsed_time(ev1) / 5

    ws = emri.Workspace()
    out = {"stat": torch.empty(n, dtype=torch.float32, device=dev),
           "topk_val": torch.empty(top_k, dtype=torch.float32, device=dev),
           "topk_idx": torch.empty(top_k, dtype=torch.int64, device=dev)}

    def step(k=top_k):
        return emri.score_tracks(spec, f0_d, U_d, C_d, k, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: exactly `steps` whole-path steps
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps

    # the scoring kernel alone (top_k = 0: per-segment constants + scoring launch)
    for _ in range(2):
        step(0)
    ev0.record()
    for _ in range(args.steps):
        step(0)
    ev1.record()
    torch.cuda.synchronize()
    ms_kernel = ev0.elapsed_time(ev1) / args.steps

    n_seg, n_bins = spec.n_seg, spec.n_bins
    evals = n * n_seg
    b_eff = n * (4 * K + 4) + evals * 4 + n_seg * n_bins * 4
    achieved = b_eff / (ms_kernel * 1e-3) / 1e9
    traffic = measured_traffic()

    line = {
        "metric": "template-segment evals/s (plain FP32 path, 1-year stream)",
        "value": evals / (ms * 1e-3),
        "unit": "template-segment evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded coloured Gaussian noise + one chirp at SNR 30; seeded uniform coefficients in the basis box)",
        "config": {"workload": "one-year stream: 3.15e7 s at 10 s, SFT 16384 samples, 192 segments x 8193 bins, "
                               "FP32 power; K=8 basis from 5000 chirp tracks; 1e7 templates; top-256",
                   "templates": n, "segments": n_seg, "bins": n_bins, "K": K, "top_k": top_k,
                   "positions": "f64", "power": "f32", "statistic": "f32 runs of 8, f64 across"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "score_fast_kernel<K=8, TPL=5, f32> (1024 threads)",
                     "kernel_ms": ms_kernel, "algorithmic_bytes_per_launch": b_eff},
        "cpu_baseline": cpu,
        "one_off": {"build_sfts_ms": t_sfts_ms, "build_basis_s": t_basis},
        "h2d_coefficients_s": t_h2d,
        "end_to_end_with_h2d_evals_per_s": evals / (ms * 1e-3 + t_h2d),
        "topk_ms": ms - ms_kernel,
    }
    forms = [f for f in args.forms.split(",") if f and f != "none"]
    if forms:
        del out, C_d
        torch.cuda.empty_cache()
        runners = {"precision": lambda: precision_form(st), "batched": batched_form,
                   "serving": lambda: serving_form(args.serve_seconds), "search": search_form,
                   "harmonics": lambda: harmonics_form(st), "chirp": lambda: chirp_form(st)}
        line["forms"] = {f: runners[f]() for f in forms}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
