"""Autotuner for the batched form: pick the tile shape of a persistent batched
launch by timing every compiled option on the batch itself.

A tile option is (rows_per_step, templates_per_lane):

* rows_per_step -- spectrogram rows staged in LDS per pipeline step (1, 2 or
  4; more rows per step mean fewer workgroup barriers but need the rows of a
  step, twice, in LDS);
* templates_per_lane -- templates each lane keeps in registers (the tile is
  templates_per_lane x 512 templates per workgroup); the library lists the
  values it compiled for K (score_batched_tile_options).

Every feasible option is planned and replayed with HIP events on the caller's
stream; the fastest (median of ``repeats`` runs) wins.  Results are cached in
a JSON file keyed by the device and a coarse signature of the batch (K, power
type, precision, problem count, log2 of the total templates and of the
largest row, median segment count), so a serving loop or a repeated search
tunes each batch shape once.
"""
from __future__ import annotations

import json
import math
import os
import statistics
from dataclasses import dataclass

from . import BatchPlan, EmriError, Workspace, batched_tile_options

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "emri_autotune.json")


@dataclass
class TuneResult:
    rows_per_step: int
    templates_per_lane: int
    ms: float
    table: list            # [(rows_per_step, templates_per_lane, median ms or None if infeasible)]
    cached: bool = False


def signature(problems, K: int, precision: str) -> str:
    """Coarse shape key of a batch (problems with similar shapes share a tuning)."""
    import torch
    n_tmpl = sum(int(pb.coeffs.shape[0]) for pb in problems)
    n_seg = sorted(pb.spec.n_seg for pb in problems) or [0]
    max_row = max((pb.spec.row_pitch * pb.spec.data.element_size() for pb in problems), default=0)
    dtype = problems[0].spec.data.dtype if problems else torch.float32
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return "|".join(str(x) for x in (
        dev, K, str(dtype).replace("torch.", ""), precision, len(problems),
        int(math.log2(max(n_tmpl, 1))), int(math.log2(max(max_row, 1))), n_seg[len(n_seg) // 2]))


def candidates(K: int, precision: str) -> list:
    """Tile options to try: every rows_per_step x every compiled templates_per_lane."""
    if precision == "mixed":
        return [(4, 0)]                       # one compiled shape: 4 rows per round of products
    return [(g, t) for g in (4, 2, 1) for t in batched_tile_options(K)]


def _time_plan(plan, stream, repeats: int) -> float:
    import torch
    plan.run(stream)                          # warm up (and first-touch the outputs)
    times = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.run(stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, cache: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass                                  # a read-only cache location only costs re-tuning


def tune(problems, K: int, precision: str = "plain", repeats: int = 5, cache_path: str | None = DEFAULT_CACHE,
         force: bool = False, stream=None) -> TuneResult:
    """Fastest tile option for this batch (from the cache unless ``force``)."""
    import torch
    stream = stream or torch.cuda.current_stream()
    key = signature(problems, K, precision)
    cache = _load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        c = cache[key]
        return TuneResult(c["rows_per_step"], c["templates_per_lane"], c["ms"], c["table"], cached=True)
    ws = Workspace()
    table = []
    for rows, tpl in candidates(K, precision):
        try:
            plan = BatchPlan(problems, K, rows_per_step=rows, templates_per_lane=tpl, precision=precision,
                             workspace=ws, stream=stream)
        except EmriError as e:
            if e.status != -5:                # EUNSUPPORTED: this option does not fit these rows
                raise
            table.append((rows, tpl, None))
            continue
        table.append((rows, tpl, _time_plan(plan, stream, repeats)))
    timed = [t for t in table if t[2] is not None]
    if not timed:
        raise RuntimeError("no tile option is feasible for this batch")
    rows, tpl, ms = min(timed, key=lambda t: t[2])
    if cache_path:
        cache[key] = {"rows_per_step": rows, "templates_per_lane": tpl, "ms": ms, "table": table}
        _store_cache(cache_path, cache)
    return TuneResult(rows, tpl, ms, table)


def tuned_plan(problems, K: int, precision: str = "plain", workspace=None, stream=None, **kw) -> tuple:
    """(BatchPlan with the tuned tile option, TuneResult)."""
    res = tune(problems, K, precision, stream=stream, **kw)
    plan = BatchPlan(problems, K, rows_per_step=res.rows_per_step, templates_per_lane=res.templates_per_lane,
                     precision=precision, workspace=workspace, stream=stream)
    return plan, res
