"""The linear-chirp statistic (Sec. II B, Eqs. (4)-(7)) on the GPU against the FP64 oracle.

Bars (from the arithmetic): complex SFTs within one FP32 rounding of the
oracle's FP64 values (plus 1e-13 of the row's largest magnitude); the
statistic within 1e-4 relative per template (the GPU evaluates the template
as a 256-point FP32 DFT of samples whose phases come from a short product
recurrence, within ~1e-5 of the continuum template, and sums in FP32 trees:
its error on S is ~1e-6 typical and up to ~2e-5 over 1e6 one-year
templates, larger only where a segment's inner product nearly cancels,
which carries little weight in the sum); segment validity decided
identically.
"""
import numpy as np
import pytest

import oracle
import oracle.chirp as och
import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n_sft", [60, 8640, 16384])
def test_complex_sfts_match_oracle(gpu_lib, n_sft):
    import torch
    emri = gpu_lib
    g = np.random.default_rng(n_sft + 1)
    dt, n_seg = 10.0, 5
    x = g.standard_normal(n_seg * n_sft + 7) * 3.0
    n_bins = n_sft // 2 + 1
    psd = g.uniform(10.0, 30.0, n_bins)
    psd[0] = np.inf
    psd[n_bins // 3] = 0.0
    spec = emri.build_sfts(_t(x), dt, n_sft, _t(psd), dtype="c32")
    torch.cuda.synchronize()
    got = _np(spec.data)
    assert np.all(got[:, n_bins:] == 0)
    got = got[:, :n_bins].astype(np.complex128)
    ref = och.build_sfts_complex(x, dt, n_sft, psd)
    tol = 2.0 ** -23 * np.abs(ref) + 1e-13 * np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(got.real - ref.real) <= tol) and np.all(np.abs(got.imag - ref.imag) <= tol)
    assert np.all(got[:, 0] == 0) and np.all(got[:, n_bins // 3] == 0)


def _chirp_case(st, K, n, seed):
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], K)
    C = synth.coefficients(9, seed, n, lo, hi)
    return f0, U, C


def _compare(emri, st, spec, f0, U, C, top_k, rows=None, oracle_result=None, **kw):
    """GPU statistic against the oracle's (computed here, or given: the
    oracle's uncut per-segment values masked by its own validity at the cuts
    in kw)."""
    import torch
    res = emri.score_tracks_chirp(spec, _t(st["psd"]), _t(f0), _t(U), _t(C), top_k, **kw)
    torch.cuda.synchronize()
    stat = _np(res["stat"])
    rows = np.arange(C.shape[0]) if rows is None else rows
    if oracle_result is None:
        Z = _np(spec.data)[:, :spec.n_bins].astype(np.complex128)
        isq = och.inverse_sqrt_psd(st["psd"])
        okw = {k: kw[k] for k in ("p_half", "f_min", "fdot_min") if k in kw}
        o = och.score_chirp(Z, isq, f0, U, C[rows], spec.t_sft, **okw)
        want = o["stat"]
    else:
        o = oracle_result
        f = oracle.track_positions(f0, U, C[rows], 1.0)
        fd, fdd = och.track_derivatives(f, spec.t_sft)
        valid = och.segment_valid(f, fd, fdd, spec.t_sft, kw.get("f_min", och.F_MIN), kw.get("fdot_min", och.FDOT_MIN))
        want = np.where(valid, o["per_segment"], 0.0).sum(axis=1)
    rel = np.abs(stat[rows] - want) / np.maximum(np.abs(want), 1e-30)
    assert rel.max() <= 1e-4, (rel.max(), np.argmax(rel))
    return res, stat, o


def test_chirp_statistic_matches_oracle_config0(gpu_lib):
    """Config-0 stream (30 segments x 4321 bins, white noise + a chirp), K = 4,
    60 templates in the box plus the injection's own projection; the oracle
    reads the GPU's complex SFTs (checked against the oracle's above)."""
    import torch
    emri = gpu_lib
    st = synth.stream_config0()
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="c32")
    torch.cuda.synchronize()
    f0, U, C = _chirp_case(st, 4, 60, 1)
    inj = st["injection"]
    f_true = synth.chirp_frequency(st["t_mid"], inj["f0"], inj["tau"])
    C = np.concatenate([((f_true - f0) @ U).astype(np.float32)[None, :], C])
    res, stat, o = _compare(emri, st, spec, f0, U, C, 8)
    assert int(_np(res["topk_idx"])[0]) == 0             # the injection ranks first
    assert np.array_equal(_np(res["topk_val"]), stat[_np(res["topk_idx"])])


@pytest.mark.parametrize("p_half", [0, 1, 37, 100])
def test_chirp_half_widths_and_cuts(gpu_lib, p_half):
    import torch
    emri = gpu_lib
    st = synth.stream_config0()
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="c32")
    torch.cuda.synchronize()
    f0, U, C = _chirp_case(st, 4, 30, 2)
    C[:5] = C[:5] * 40.0                                   # far outside the box: cuts and out-of-row bins
    C[5] = np.nan
    Z = _np(spec.data)[:, :spec.n_bins].astype(np.complex128)
    o = och.score_chirp(Z, och.inverse_sqrt_psd(st["psd"]), f0, U, C, spec.t_sft, p_half=p_half,
                        f_min=-np.inf, fdot_min=-np.inf)
    for f_min, fdot_min in ((-np.inf, -np.inf), (3e-3, 0.0), (10 ** -3.5, 1e-13)):
        _compare(emri, st, spec, f0, U, C, 0, oracle_result=o, p_half=p_half, f_min=f_min, fdot_min=fdot_min)
    if p_half == 0:
        # one bin: the nearest-bin power of build_sfts, summed over the valid segments
        P = oracle.build_sfts(st["x"], st["dt"], st["n_sft"], st["psd"])
        res = emri.score_tracks_chirp(spec, _t(st["psd"]), _t(f0), _t(U), _t(C), 0, p_half=0,
                                      f_min=-np.inf, fdot_min=-np.inf)
        torch.cuda.synchronize()
        f = oracle.track_positions(f0, U, C, 1.0)
        fd, fdd = och.track_derivatives(f, spec.t_sft)
        valid = och.segment_valid(f, fd, fdd, spec.t_sft, -np.inf, -np.inf)
        b, inrow = oracle.chosen_bins(f * spec.t_sft, P.shape[1])
        want = np.where(valid & inrow, P[np.arange(P.shape[0])[None, :], np.where(inrow, b, 0)], 0.0).sum(axis=1)
        got = _np(res["stat"])
        assert np.allclose(got, want, rtol=1e-5, atol=0)


@pytest.mark.parametrize("p_half", [37, 100])
def test_chirp_psd_weighting(gpu_lib, p_half):
    """A PSD that changes from bin to bin (uniform in [1, 40]) over twelve
    segments holding a noisy linear chirp: the 1/S weighting of every window
    bin matters here (a kernel that ignored it, or read the weights wrongly,
    would be off by 2-46 %)."""
    import torch
    emri = gpu_lib
    g = np.random.default_rng(21)
    n_sft, dt, n_seg, K = 2048, 5.0, 12, 3
    n_bins = n_sft // 2 + 1
    T = n_sft * dt
    psd = g.uniform(1.0, 40.0, n_bins)
    x = g.standard_normal(n_sft * n_seg) * 3.0
    t = np.arange(x.size) * dt
    x += 0.8 * np.cos(2 * np.pi * (300.3 / T) * t + np.pi * (2.0 / T ** 2) * t * t)
    spec = emri.build_sfts(_t(x), dt, n_sft, _t(psd), dtype="c32")
    torch.cuda.synchronize()
    tm = (np.arange(n_seg) + 0.5) * T
    f0 = (300.3 + 2.0 * tm / T) / T
    v = (tm - tm.mean()) / T / n_seg
    U = np.stack([np.ones(n_seg), v, v * v], axis=1) * (4.0 / T)
    C = g.uniform(-2, 2, (40, K)).astype(np.float32)
    _compare(emri, {"psd": psd}, spec, f0, U, C, 5, p_half=p_half, f_min=-np.inf, fdot_min=-np.inf)


@pytest.mark.parametrize("n_seg,K", [(1, 2), (2, 2), (3, 1), (3, 0), (64, 2), (65, 3), (130, 2)])
def test_chirp_segment_counts_and_K(gpu_lib, n_seg, K):
    """One and two segments (the derivatives' special cases), three, a full
    64-segment chunk, a ragged second chunk, K = 0 (every template is f0);
    P = 10, cut-offs off; against the oracle; an empty batch is accepted."""
    import torch
    emri = gpu_lib
    g = np.random.default_rng(500 + n_seg + K)
    n_sft, dt = 512, 2.0
    T = n_sft * dt
    psd = g.uniform(5.0, 15.0, n_sft // 2 + 1)
    x = g.standard_normal(n_sft * n_seg)
    spec = emri.build_sfts(_t(x), dt, n_sft, _t(psd), dtype="c32")
    torch.cuda.synchronize()
    f0 = g.uniform(60.0, 190.0, n_seg) / T
    U = g.standard_normal((n_seg, K)) * (3.0 / T)
    C = g.uniform(-2, 2, (33, K)).astype(np.float32)
    _compare(emri, {"psd": psd}, spec, f0, U, C, 4, p_half=10, f_min=-np.inf, fdot_min=-np.inf)
    res = emri.score_tracks_chirp(spec, _t(psd), _t(f0), _t(U), _t(C[:0]), 0, p_half=10)
    torch.cuda.synchronize()
    assert res["stat"].numel() == 0


def test_chirp_one_year_sampled(gpu_lib):
    """The one-year complex SFTs (192 segments x 8193 bins), K = 8, 2e5 templates in
    the box, P = 100: 8 sampled templates and the top-10 against the oracle."""
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="c32")
    torch.cuda.synchronize()
    f0, U, C = _chirp_case(st, 8, 200_000, 3)
    res = emri.score_tracks_chirp(spec, _t(st["psd"]), _t(f0), _t(U), _t(C), 10)
    torch.cuda.synchronize()
    top = _np(res["topk_idx"])
    rows = np.unique(np.concatenate([np.random.default_rng(4).integers(0, C.shape[0], 8), top]))
    _compare(emri, st, spec, f0, U, C, 10, rows=rows)
    stat = _np(res["stat"])
    assert np.array_equal(_np(res["topk_val"]), stat[top])
    order = np.lexsort((np.arange(stat.size), -stat.astype(np.float64)))[:10]
    assert np.array_equal(top, order)
