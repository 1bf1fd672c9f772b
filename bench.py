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
                      f"{cores} worker processes, {wall:.2f} s wall"}


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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--templates", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=1 << 21)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (reference for traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(templates would shard across GPUs with one top-k exchange; see the design notes)",
              file=sys.stderr)
        return 2

    # ---- inputs (host), before any GPU initialisation -------------------------------
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
        cpu = cpu_baseline(P_host, f0, U, C, st["n_sft"] * st["dt"], min(args.cpu_sample, n))

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
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        try:
            traffic = json.load(open(PROFILE_TRAFFIC)).get("hbm_bytes_per_launch")
        except (OSError, ValueError):
            traffic = None

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
                     "kernel": "score_fast_kernel<K=8, TPL=9, f32>",
                     "kernel_ms": ms_kernel, "algorithmic_bytes_per_launch": b_eff},
        "cpu_baseline": cpu,
        "one_off": {"build_sfts_ms": t_sfts_ms, "build_basis_s": t_basis},
        "h2d_coefficients_s": t_h2d,
        "end_to_end_with_h2d_evals_per_s": evals / (ms * 1e-3 + t_h2d),
        "topk_ms": ms - ms_kernel,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
