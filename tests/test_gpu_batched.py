"""Batched form on the GPU: every problem of one persistent launch gives, bit for
bit, the result of a standalone score_tracks call; the run replays correctly
from a captured HIP graph; tile options do not change any result."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def make_problems(emri, dtype, seed=0, n_specs=3, n_problems=7):
    import torch
    g = np.random.default_rng(seed)
    specs = []
    for s in range(n_specs):
        n_seg = int(g.integers(5, 40))
        n_bins = int(g.integers(300, 3000))
        t = 163840.0
        P = g.exponential(size=(n_seg, n_bins))
        f0 = g.uniform(0.2, 0.8, n_seg) * n_bins / t
        U = g.standard_normal((n_seg, 8)) * (20.0 / t)
        specs.append((emri.spectrogram_from_power(P, t, dtype), _t(f0), _t(U)))
    # a spectrogram without segments: every statistic is zero
    specs.append((emri.spectrogram_from_power(np.zeros((0, 64)), 163840.0, dtype),
                  _t(np.zeros(0)), _t(np.zeros((0, 8)))))
    probs = []
    sizes = [0, 1, 777, 4608 * 2 + 5, 20000, 9000, 3]
    for i in range(n_problems):
        spec, f0, U = specs[n_specs if i == 6 else i % n_specs]
        n = sizes[i % len(sizes)]
        C = g.uniform(-40, 40, (n, 8)).astype(np.float32)
        top_k = [0, 5, 16, 100, 256, 7, 4][i % 7]
        kmin, kmax = (0, -1) if i % 3 else (10, spec.n_bins - 20)
        probs.append(emri.Problem(spec, f0, U, _t(C), top_k=top_k, k_min=kmin, k_max=kmax))
    return probs


def standalone(emri, pb):
    import torch
    res = emri.score_tracks(pb.spec, pb.f0, pb.U, pb.coeffs, pb.top_k, k_min=pb.k_min, k_max=pb.k_max)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def check_equal(emri, probs):
    for i, pb in enumerate(probs):
        ref = standalone(emri, pb)
        assert np.array_equal(pb.stat.cpu().numpy(), ref["stat"]), i
        assert np.array_equal(pb.topk_idx.cpu().numpy(), ref["topk_idx"]), i
        assert np.array_equal(pb.topk_val.cpu().numpy(), ref["topk_val"]), i


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_batched_equals_standalone(gpu_lib, dtype):
    import torch
    emri = gpu_lib
    probs = make_problems(emri, dtype)
    plan = emri.BatchPlan(probs, 8)
    plan.run()
    torch.cuda.synchronize()
    check_equal(emri, probs)


@pytest.mark.parametrize("K", [1, 3, 4, 5, 12, 16])
@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_batched_other_K(gpu_lib, K, precision):
    """The batched kernels of other basis sizes: every problem equals its
    standalone call bit for bit, and sampled statistics match the oracle."""
    import torch
    emri = gpu_lib
    g = np.random.default_rng(40 + K)
    probs, raw = [], []
    for i, (n_seg, n_bins, n, top_k) in enumerate([(17, 1200, 6000, 32), (9, 400, 777, 5), (30, 2600, 11000, 100)]):
        t = 163840.0
        P = g.exponential(size=(n_seg, n_bins))
        spec = emri.spectrogram_from_power(P, t, "f16")
        f0 = g.uniform(0.3, 0.7, n_seg) * n_bins / t
        U = g.standard_normal((n_seg, K)) * (15.0 / t)
        C = g.uniform(-3, 3, (n, K)).astype(np.float32)
        probs.append(emri.Problem(spec, _t(f0), _t(U), _t(C), top_k=top_k))
        raw.append((spec, f0, U, C))
    emri.BatchPlan(probs, K, precision=precision).run()
    torch.cuda.synchronize()
    for pb, (spec, f0, U, C) in zip(probs, raw):
        ref = emri.score_tracks(pb.spec, pb.f0, pb.U, pb.coeffs, pb.top_k, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(pb.stat, ref["stat"])
        assert torch.equal(pb.topk_idx, ref["topk_idx"])
        rows = np.arange(0, C.shape[0], 97)
        P_used = spec.power().cpu().numpy().astype(np.float64)
        o = oracle.score_tracks(P_used, f0, U, C[rows], spec.t_sft, 0)
        got = pb.stat.cpu().numpy()[rows]
        if precision == "plain":
            # every sampled template to the plain bar; near-ties at the GPU's own bins
            val = emri.score_tracks(pb.spec, pb.f0, pb.U, _t(C[rows]), 0, want_bins=True, want_near_tie=True)
            torch.cuda.synchronize()
            assert np.array_equal(val["stat"].cpu().numpy(), got)
            gb = val["bins"].cpu().numpy().astype(np.int64)
            near = oracle.near_tie_mask(oracle.track_positions(f0, U, C[rows], spec.t_sft))
            ob = oracle.chosen_bins(oracle.track_positions(f0, U, C[rows], spec.t_sft), P_used.shape[1])
            ob = np.where(ob[1], ob[0], -1)
            assert np.all((gb == ob) | near)
            ref = oracle.score.fsum_rows(P_used, gb)
            assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) <= 1e-5
        else:
            rel = np.abs(got - o["stat"]) / np.abs(o["stat"])
            assert np.quantile(rel, 0.99) <= 2e-3


@pytest.mark.parametrize("rows,tpl", [(1, 0), (2, 0), (4, 0), (0, 6)])
def test_batched_tile_options_do_not_change_results(gpu_lib, rows, tpl):
    import torch
    emri = gpu_lib
    probs = make_problems(emri, "f16", seed=3)
    emri.BatchPlan(probs, 8).run()
    torch.cuda.synchronize()
    ref = [(p.stat.clone(), p.topk_idx.clone()) for p in probs]
    for p in probs:
        p.stat.fill_(-1.0)
    emri.BatchPlan(probs, 8, rows_per_step=rows, templates_per_lane=tpl).run()
    torch.cuda.synchronize()
    for p, (s, i) in zip(probs, ref):
        assert torch.equal(p.stat, s) and torch.equal(p.topk_idx, i)


def test_batched_graph_replay(gpu_lib):
    import torch
    emri = gpu_lib
    probs = make_problems(emri, "f32", seed=5)
    plan = emri.BatchPlan(probs, 8)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run()
    g = np.random.default_rng(11)
    for rep in range(3):
        for pb in probs:
            if pb.coeffs.shape[0]:
                pb.coeffs.copy_(_t(g.uniform(-40, 40, tuple(pb.coeffs.shape)).astype(np.float32)))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check_equal(emri, probs)


def test_batched_streams_of_config3_shape_against_oracle(gpu_lib):
    """Four uneven one-year-noise streams (N_seg 48..192) at FP16, sampled against the oracle."""
    import torch
    emri = gpu_lib
    probs, refs = [], []
    for s, months in enumerate((3.2, 6.5, 9.1, 12.0)):
        st = synth.stream_config1(stream=s, cfg=3, duration_s=months * synth.YEAR_S / 12, snr=25.0)
        spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="f16")
        f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], 8)
        C = synth.coefficients(3, s, 30000 + 5000 * s, lo, hi)
        probs.append(emri.Problem(spec, _t(f0), _t(U), _t(C), top_k=64))
        refs.append((spec, f0, U, C))
    emri.BatchPlan(probs, 8).run()
    torch.cuda.synchronize()
    for pb, (spec, f0, U, C) in zip(probs, refs):
        P16 = spec.power().cpu().numpy().astype(np.float64)
        rows = np.arange(0, C.shape[0], 37)
        o = oracle.score_tracks(P16, f0, U, C[rows], spec.t_sft, 0)
        got = pb.stat.cpu().numpy()[rows]
        near = oracle.near_tie_mask(oracle.track_positions(f0, U, C[rows], spec.t_sft)).any(axis=1)
        rel = np.abs(got - o["stat"]) / np.abs(o["stat"])
        assert rel[~near].max() <= 1e-5
