"""Mixed-precision form on the GPU (BF16-split matrix-core contraction, FP32
accumulation, FP64 offset and rounding, FP16 or FP32 power).

* exactness: when every product and partial sum is exact in FP32 the mixed
  form must choose the same bins as FP64 and return the plain statistic bit
  for bit (this pins the operand / result layout of the matrix instructions);
* accuracy on the one-year stream at its full shape, against the FP64 oracle:
  statistic relative error p99 <= 2e-3 and top-100 overlap >= 99;
* the batched form in mixed precision equals standalone calls bit for bit;
* huge or non-finite coefficients contribute nothing, as in the plain form.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def _score(emri, spec, f0, U, C, top_k=0, precision="plain", **kw):
    import torch
    res = emri.score_tracks(spec, _t(f0), _t(U), _t(np.asarray(C, dtype=np.float32)), top_k,
                            precision=precision, **kw)
    torch.cuda.synchronize()
    return {k: _np(v) for k, v in res.items()}


@pytest.mark.parametrize("K", [1, 3, 4, 5, 8, 12, 16])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_mixed_exact_inputs_equal_plain(gpu_lib, K, dtype):
    emri = gpu_lib
    g = np.random.default_rng(100 + K)
    n_seg, n_bins, t = 23, 700, 1.0
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, dtype)
    f0 = np.round(g.uniform(250, 450, n_seg)) + 0.25          # fraction 1/4: never a tie
    U = g.integers(-3, 4, (n_seg, K)).astype(np.float64)       # exact in BF16
    C = (g.integers(-16, 17, (5000, K)) / 2.0).astype(np.float32)   # halves: products exact
    plain = _score(emri, spec, f0, U, C, 32)
    mixed = _score(emri, spec, f0, U, C, 32, precision="mixed")
    assert np.array_equal(plain["stat"], mixed["stat"])
    assert np.array_equal(plain["topk_idx"], mixed["topk_idx"])
    # and both are the oracle's statistic
    o = oracle.score_tracks(_np(spec.power()).astype(np.float64), f0, U, C, t, 0)
    assert np.max(np.abs(plain["stat"] - o["stat"]) / np.maximum(o["stat"], 1e-30)) <= 1e-5


@pytest.mark.parametrize("K", [4, 8, 16])
@pytest.mark.parametrize("n_seg", [1, 2, 3, 5, 6, 7, 8, 9, 10, 11, 12])
def test_mixed_short_and_ragged_segment_counts(gpu_lib, K, n_seg):
    """Every position of the last staging step (4 segments) and of the last
    loop turn (two steps), with one and two segments of gathers in flight
    (K = 4 and 16: one; K = 8: two); 14 workgroups of 500 templates each, so
    the half-size tail tile and its idle lanes too."""
    emri = gpu_lib
    g = np.random.default_rng(1000 + 17 * K + n_seg)
    n_bins, t = 600, 1.0
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, "f16")
    f0 = np.round(g.uniform(200, 400, n_seg)) + 0.25
    U = g.integers(-3, 4, (n_seg, K)).astype(np.float64)
    C = (g.integers(-16, 17, (7000, K)) / 2.0).astype(np.float32)
    plain = _score(emri, spec, f0, U, C, 16)
    mixed = _score(emri, spec, f0, U, C, 16, precision="mixed")
    assert np.array_equal(plain["stat"], mixed["stat"])
    assert np.array_equal(plain["topk_idx"], mixed["topk_idx"])
    o = oracle.score_tracks(_np(spec.power()).astype(np.float64), f0, U, C, t, 0)
    assert np.max(np.abs(mixed["stat"] - o["stat"]) / np.maximum(o["stat"], 1e-30)) <= 1e-5


def test_mixed_three_piece_split_beats_one_piece(gpu_lib):
    """Coefficients and U with 24 significant bits: a one-piece (plain BF16) product
    would move most tracks by many bins; the split keeps almost every bin."""
    emri = gpu_lib
    g = np.random.default_rng(7)
    n_seg, n_bins, t, K = 40, 4000, 1.0, 8
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, "f16")
    f0 = g.uniform(1500, 2500, n_seg)
    U = g.standard_normal((n_seg, K)) * 40.0
    C = g.uniform(-10, 10, (20000, K)).astype(np.float32)
    mixed = _score(emri, spec, f0, U, C, 0, precision="mixed")
    plain = _score(emri, spec, f0, U, C, 0)
    P16 = _np(spec.power()).astype(np.float64)
    o = oracle.score_tracks(P16, f0, U, C, t, 0)
    rel = np.abs(mixed["stat"] - o["stat"]) / o["stat"]
    assert np.mean(mixed["stat"] == plain["stat"]) > 0.9      # every bin the same as FP64
    assert np.quantile(rel, 0.99) <= 2e-3
    # the same positions rounded through one BF16 piece each
    bf = lambda a: (np.asarray(a, np.float32).view(np.uint32) + 0x8000 & 0xFFFF0000).view(np.float32)
    x1 = f0[None, :] + bf(C) @ bf(U).T
    assert np.mean(np.rint(x1) != np.rint(oracle.track_positions(f0, U, C, t))) > 0.3


def test_mixed_one_year_full_size_error_report(gpu_lib):
    """1e7 templates, K = 8, FP16 power: statistic error against the FP64 oracle (on the same
    FP16 power) on sampled templates, and the top-100 overlap on the first 2e5 templates."""
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], 8)
    n = st["n_tmpl"]
    C = synth.coefficients(1, 0, n, lo, hi)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="f16")
    res = emri.score_tracks(spec, _t(f0), _t(U), _t(C), 0, precision="mixed")
    torch.cuda.synchronize()
    stat = _np(res["stat"])
    P16 = _np(spec.power()).astype(np.float64)
    rows = np.random.default_rng(3).integers(0, n, 30000)
    o = oracle.score_tracks(P16, f0, U, C[rows], spec.t_sft, 0)
    rel = np.abs(stat[rows] - o["stat"]) / np.abs(o["stat"])
    assert np.quantile(rel, 0.99) <= 2e-3, np.quantile(rel, [0.5, 0.99, 1.0])
    m = 200_000
    o2 = oracle.score_tracks(P16, f0, U, C[:m], spec.t_sft, 100)
    sub = emri.score_tracks(spec, _t(f0), _t(U), _t(C[:m]), 100, precision="mixed")
    torch.cuda.synchronize()
    overlap = len(set(_np(sub["topk_idx"]).tolist()) & set(o2["topk_idx"].tolist()))
    assert overlap >= 99


def test_mixed_batched_equals_standalone(gpu_lib):
    import torch
    emri = gpu_lib
    g = np.random.default_rng(9)
    probs = []
    for i, (n_seg, n_bins, n) in enumerate([(13, 900, 7000), (30, 2500, 1), (4, 300, 12345), (21, 1500, 0),
                                            (30, 2500, 5000)]):
        t = 2000.0
        P = g.exponential(size=(n_seg, n_bins))
        spec = emri.spectrogram_from_power(P, t, "f16")
        f0 = g.uniform(0.3, 0.7, n_seg) * n_bins / t
        U = g.standard_normal((n_seg, 8)) * (30.0 / t)
        C = g.uniform(-5, 5, (n, 8)).astype(np.float32)
        probs.append(emri.Problem(spec, _t(f0), _t(U), _t(C), top_k=[16, 3, 100, 5, 0][i]))
    emri.BatchPlan(probs, 8, precision="mixed").run()
    torch.cuda.synchronize()
    for pb in probs:
        ref = emri.score_tracks(pb.spec, pb.f0, pb.U, pb.coeffs, pb.top_k, precision="mixed")
        torch.cuda.synchronize()
        assert torch.equal(pb.stat, ref["stat"])
        assert torch.equal(pb.topk_idx, ref["topk_idx"])


def test_mixed_wild_coefficients(gpu_lib):
    emri = gpu_lib
    g = np.random.default_rng(11)
    n_seg, n_bins, t, K = 9, 500, 1.0, 4
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, "f16")
    f0 = g.uniform(200, 300, n_seg)
    U = g.standard_normal((n_seg, K))
    C = g.uniform(-5, 5, (3000, K)).astype(np.float32)
    C[5] = [np.nan, 0, 0, 0]
    C[6] = [np.inf, 1, 0, 0]
    C[7] = [3e38, -3e38, 1, 1]
    C[8] = [1e9, 0, 0, 0]
    mixed = _score(emri, spec, f0, U, C, 0, precision="mixed")
    plain = _score(emri, spec, f0, U, C, 0)
    assert np.all(mixed["stat"][5:9] == 0) and np.all(plain["stat"][5:9] == 0)
    ok = np.ones(3000, bool)
    ok[5:9] = False
    rel = np.abs(mixed["stat"][ok] - plain["stat"][ok]) / plain["stat"][ok]
    assert np.quantile(rel, 0.99) <= 2e-3
