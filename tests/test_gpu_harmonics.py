"""Multi-harmonic form (Sec. IV) on the GPU against the FP64 oracle.

Bars: with one harmonic of ratio 1 the statistic is score_tracks' bit for
bit (same positions, rounding and summation order); otherwise every template
within 1e-5 relative of the oracle, where a template with a harmonic
position within 1e-6 bin of a half-integer may take either neighbour there
(every such combination is tried); top-k as a set, up to entries within
2e-5 of the k-th value.
"""
import itertools

import numpy as np
import pytest

import oracle
import oracle.harmonics as ohm
import synth
from tests.test_gpu_parity import check_topk

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def score_harm(emri, spec, f0, U, C, ratios, top_k=0, **kw):
    import torch
    res = emri.score_tracks_harmonics(spec, _t(f0), _t(U), _t(np.asarray(C, np.float32)), ratios, top_k, **kw)
    torch.cuda.synchronize()
    return {k: _np(v) for k, v in res.items()}


def check_harmonics(P, f0, U, C, t, ratios, gpu_stat, k_min=0, k_max=None, rows=None):
    """Every (sampled) template against the oracle; near-tie templates may take either neighbour."""
    rows = np.arange(C.shape[0]) if rows is None else rows
    o = ohm.score_harmonics(P, f0, U, C[rows], t, ratios, 0, k_min, k_max)
    got = gpu_stat[rows]
    rel = np.abs(got - o["stat"]) / np.maximum(np.abs(o["stat"]), 1e-30)
    ok = ~o["near"]
    assert rel[ok].max() <= 1e-5, rel[ok].max()
    n_bins = P.shape[1]
    kmax = n_bins - 1 if k_max is None else k_max
    x = oracle.track_positions(f0, U, C[rows], t)
    for jj in np.flatnonzero(o["near"]):
        xh = ohm.harmonic_positions(x[jj:jj + 1], ratios)[:, 0, :]          # (H, n_seg)
        base = 0.0
        alts = []
        for h in range(xh.shape[0]):
            for a in range(xh.shape[1]):
                v = xh[h, a]
                near = abs(v - np.floor(v) - 0.5) < oracle.NEAR_TIE_BAND
                cands = [int(np.floor(v)), int(np.floor(v)) + 1] if near else [int(np.rint(v))]
                vals = [P[a, b] if k_min <= b <= kmax else 0.0 for b in cands]
                if near:
                    alts.append(vals)
                else:
                    base += vals[0]
        assert len(alts) <= 8
        sums = [base + sum(c) for c in itertools.product(*alts)]
        assert min(abs(got[jj] - s_) / max(abs(s_), 1e-30) for s_ in sums) <= 1e-5, (jj, got[jj], sums)
    return o


@pytest.mark.parametrize("K", [1, 4, 8, 16])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_one_harmonic_of_ratio_one_is_score_tracks(gpu_lib, K, dtype):
    emri = gpu_lib
    g = np.random.default_rng(300 + K)
    n_seg, n_bins, t = 21, 2500, 1000.0
    spec = emri.spectrogram_from_power(g.exponential(size=(n_seg, n_bins)), t, dtype)
    f0 = g.uniform(0.3, 0.7, n_seg) * n_bins / t
    U = g.standard_normal((n_seg, K)) * (40.0 / t)
    C = g.uniform(-3, 3, (40_000, K)).astype(np.float32)
    import torch
    ref = emri.score_tracks(spec, _t(f0), _t(U), _t(C), 50)
    torch.cuda.synchronize()
    h = score_harm(emri, spec, f0, U, C, [1.0], 50)
    assert np.array_equal(h["stat"], _np(ref["stat"]))
    assert np.array_equal(h["topk_idx"], _np(ref["topk_idx"]))


@pytest.mark.parametrize("K,ratios", [(1, (1.0, 0.5)), (3, (1.0, 0.5, 1.5)), (8, (1.0, 0.5, 1.5, 2.0)),
                                      (16, (1.0, 1.5)), (8, (0.75, 1.25, 3.0))])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_harmonics_match_oracle(gpu_lib, K, ratios, dtype):
    emri = gpu_lib
    g = np.random.default_rng(400 + K + len(ratios))
    n_seg, n_bins, t = 19, 3000, 1000.0
    spec = emri.spectrogram_from_power(g.exponential(size=(n_seg, n_bins)), t, dtype)
    P = _np(spec.power()).astype(np.float64)
    f0 = g.uniform(0.2, 0.6, n_seg) * n_bins / t
    U = g.standard_normal((n_seg, K)) * (60.0 / t)
    n = 30_011                                              # ragged: several tiles, a partial last one
    C = g.uniform(-3, 3, (n, K)).astype(np.float32)
    res = score_harm(emri, spec, f0, U, C, ratios, 40)
    o = check_harmonics(P, f0, U, C, t, ratios, res["stat"])
    ref = o["stat"].copy()
    check_topk(res["topk_val"], res["topk_idx"], np.where(o["near"], res["stat"], ref), 40)


def test_harmonics_bin_range_and_wild(gpu_lib):
    emri = gpu_lib
    g = np.random.default_rng(5)
    n_seg, n_bins, t, K = 9, 800, 10.0, 4
    spec = emri.spectrogram_from_power(g.exponential(size=(n_seg, n_bins)), t, "f32")
    P = _np(spec.power()).astype(np.float64)
    f0 = g.uniform(20.0, 40.0, n_seg)
    U = g.standard_normal((n_seg, K))
    C = g.uniform(-3, 3, (5000, K)).astype(np.float32)
    C[3] = [np.nan, 0, 0, 0]
    C[4] = [np.inf, 0, 0, 0]
    C[5] = [3e38, 1, 1, 1]
    C[6] = [1e8, 0, 0, 0]
    ratios = (1.0, 0.5, 1.5)
    for k_min, k_max in ((0, None), (150, 500), (0, 100)):
        res = score_harm(emri, spec, f0, U, C, ratios, 0, k_min=k_min, k_max=-1 if k_max is None else k_max)
        assert np.all(res["stat"][3:7] == 0.0)
        check_harmonics(P, f0, U, C, t, ratios, res["stat"], k_min, k_max)


def test_harmonics_one_year_sampled(gpu_lib):
    """The one-year stream, 1e7 templates, K = 8, harmonics 1, 1/2, 3/2: sampled
    templates and the top-256 against the oracle."""
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], 8)
    n = st["n_tmpl"]
    C = synth.coefficients(1, 0, n, lo, hi)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]))
    ratios = (1.0, 0.5, 1.5)
    res = emri.score_tracks_harmonics(spec, _t(f0), _t(U), _t(C), ratios, 256)
    torch.cuda.synchronize()
    stat = _np(res["stat"])
    P = _np(spec.power()).astype(np.float64)
    top_idx, top_val = _np(res["topk_idx"]), _np(res["topk_val"])
    assert np.array_equal(top_val, stat[top_idx])
    g = np.random.default_rng(2)
    check_harmonics(P, f0, U, C, spec.t_sft, ratios, stat,
                    rows=np.unique(np.concatenate([g.integers(0, n, 10000), top_idx])))
    kth = float(top_val[-1])
    cand = np.flatnonzero(stat >= kth - 3e-5 * abs(kth))
    assert cand.size < 200_000
    o = ohm.score_harmonics(P, f0, U, C[cand], spec.t_sft, ratios, 0)
    ref = np.full(n, -np.inf)
    ref[cand] = np.where(o["near"], stat[cand], o["stat"])
    check_topk(top_val, top_idx, ref, 256)
