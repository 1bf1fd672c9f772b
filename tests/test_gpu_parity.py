"""Parity of the HIP path against the FP64 oracle (MI355X only).

Bars: chosen bins bit-exact except where the oracle's position lies within
1e-6 bin of a half-integer (then either neighbour is accepted and the oracle's
statistic is recomputed at the GPU's bin); statistic within 1e-5 relative;
top-k equal as a set except entries within 2e-5 of the k-th value; integer
outputs (indices, counts, bins) exact.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import pins

pytestmark = pytest.mark.gpu

STAT_RTOL = 1e-5


def _t(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _np(t):
    return t.detach().cpu().numpy()


def score_gpu(emri, P, f0, U, C, t_sft, top_k, dtype="f32", **kw):
    import torch
    spec = emri.spectrogram_from_power(np.asarray(P), t_sft, dtype)
    K = U.shape[1]
    C = np.asarray(C, dtype=np.float32)
    assert C.ndim == 2 and C.shape[1] == K
    res = emri.score_tracks(spec, _t(f0, torch.float64), _t(np.asarray(U).reshape(len(f0), K), torch.float64),
                            _t(C), top_k, **kw)
    torch.cuda.synchronize()
    return {k: _np(v) for k, v in res.items()}


def check_against_oracle(P_used, f0, U, C, t_sft, gpu, o, k_min=0, k_max=None):
    """Bins exact outside the near-tie band; S within STAT_RTOL (recomputed at GPU bins on ties)."""
    x = oracle.track_positions(f0, U, C, t_sft)
    near = oracle.near_tie_mask(x)
    gb = gpu["bins"].astype(np.int64)
    ob = o["bins"].astype(np.int64)
    mism = gb != ob
    assert not np.any(mism & ~near), np.argwhere(mism & ~near)[:5]
    if np.any(mism):
        # either neighbour of a near-tie is fine
        lo = np.floor(x[mism]).astype(np.int64)
        cand = gb[mism]
        n_bins = P_used.shape[1]
        kmax = n_bins - 1 if k_max is None else k_max
        valid_lo = np.where((lo >= k_min) & (lo <= kmax), lo, -1)
        valid_hi = np.where((lo + 1 >= k_min) & (lo + 1 <= kmax), lo + 1, -1)
        assert np.all((cand == valid_lo) | (cand == valid_hi))
    ref = oracle.score.fsum_rows(P_used, gb) if np.any(mism) else o["stat"]
    rel = np.abs(gpu["stat"] - ref) / np.maximum(np.abs(ref), 1e-30)
    assert rel.max() <= STAT_RTOL, rel.max()
    assert int(gpu["n_near_tie"][0]) == o["n_near_tie"]


def check_topk(gpu_vals, gpu_idx, stat_ref, k, tol=2e-5):
    """GPU top-k equals the exact top-k of the reference statistic, up to near-equal entries."""
    n = stat_ref.size
    kk = min(k, n)
    ov, oi = oracle.topk_order(stat_ref, k)
    assert np.all(gpu_idx[kk:] == -1) and np.all(np.isneginf(gpu_vals[kk:]))
    if kk == 0:
        return
    kth = ov[kk - 1]
    band = tol * max(abs(kth), 1e-30)
    sure = set(oi[:kk][ov[:kk] > kth + band].tolist())
    got = set(gpu_idx[:kk].tolist())
    assert sure <= got
    for j in got - sure:
        assert abs(stat_ref[j] - kth) <= band or stat_ref[j] >= kth - band
    # values are sorted and belong to their indices
    assert np.all(np.diff(gpu_vals[:kk]) <= 0)


# ------------------------------------------------------------------------ build_sfts


@pytest.mark.parametrize("n_sft", [12, 14, 30, 60, 8640, 16384])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_build_sfts_matches_oracle(gpu_lib, n_sft, dtype):
    import torch
    emri = gpu_lib
    g = np.random.default_rng(n_sft)
    dt = 10.0
    n_seg = 7 if n_sft > 100 else 5
    x = g.standard_normal(n_seg * n_sft + n_sft // 3) * 2.0
    n_bins = n_sft // 2 + 1
    psd = np.full(n_bins, 2.0 * 4.0 * dt)
    psd[0] = np.inf
    psd[n_bins // 3] = 0.0
    psd[n_bins // 2] = -1.0
    spec = emri.build_sfts(_t(x), dt, n_sft, _t(psd), dtype=dtype)
    torch.cuda.synchronize()
    assert spec.n_seg == n_seg and spec.n_bins == n_bins and spec.t_sft == n_sft * dt
    got = _np(spec.data).astype(np.float64)
    assert np.all(got[:, n_bins:] == 0.0)
    ref = oracle.build_sfts(x, dt, n_sft, psd)
    got = got[:, :n_bins]
    if dtype == "f32":
        want = ref.astype(np.float32).astype(np.float64)
        tol = 2.0 ** -23 * np.abs(ref) + 1e-13 * ref.max(axis=1, keepdims=True)
    else:
        want = ref.astype(np.float16).astype(np.float64)
        tol = 2.0 ** -10 * np.abs(ref) + 2.0 ** -24 + 1e-13 * ref.max(axis=1, keepdims=True)
    assert np.all(np.abs(got - want) <= tol), np.abs(got - want).max()
    for b in (0, n_bins // 3, n_bins // 2):
        assert np.all(got[:, b] == 0.0)


def test_build_sfts_one_year_coloured(gpu_lib):
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]))
    torch.cuda.synchronize()
    ref = oracle.build_sfts(st["x"], st["dt"], st["n_sft"], st["psd"])
    assert spec.n_seg == 192 and spec.n_bins == 8193
    got = _np(spec.power()).astype(np.float64)
    err = np.abs(got - ref.astype(np.float32))
    assert np.all(err <= 2.0 ** -23 * np.abs(ref) + 1e-12 * ref.max(axis=1, keepdims=True))


# ------------------------------------------------------------------------ score_tracks


def test_tiny_exact_cases(gpu_lib):
    for seed in range(6):
        P, f0, U, C, t = pins.tiny_score_case(seed)
        P32 = P.astype(np.float32).astype(np.float64)
        s_exact, b_exact = oracle.score_tracks_exact(P32, f0, U, C, t)
        gpu = score_gpu(gpu_lib, P32, f0, U, C, t, 3, want_bins=True, want_near_tie=True)
        assert np.array_equal(gpu["bins"], b_exact), seed
        assert np.allclose(gpu["stat"], s_exact, rtol=1e-6, atol=0)


def test_half_even_and_edges(gpu_lib):
    n_seg, n_bins, t = 6, 32, 8.0
    P = np.arange(n_seg * n_bins, dtype=np.float64).reshape(n_seg, n_bins) + 1.0
    U = np.ones((n_seg, 1))
    C = np.zeros((1, 1), np.float32)
    f0 = np.array([2.5, 3.5, 4.5, 10.5, 11.5, 0.5]) / t
    gpu = score_gpu(gpu_lib, P, f0, U, C, t, 1, want_bins=True, want_near_tie=True)
    assert list(gpu["bins"][0]) == [2, 4, 4, 10, 12, 0]
    assert int(gpu["n_near_tie"][0]) == 6
    f0b = np.array([-0.5, n_bins - 0.5, -1.5, 1.0, 2.0, n_bins - 1.0]) / t
    gpu = score_gpu(gpu_lib, P, f0b, U, C, t, 1, want_bins=True, want_near_tie=True)
    assert list(gpu["bins"][0]) == [0, -1, -1, 1, 2, n_bins - 1]
    want = P[0, 0] + P[3, 1] + P[4, 2] + P[5, n_bins - 1]
    assert gpu["stat"][0] == np.float32(want)


@pytest.mark.parametrize("k_range", [(0, None), (5, 40), (0, 17), (31, 31), (1, 63)])
def test_bin_range_and_nonfinite(gpu_lib, k_range):
    g = np.random.default_rng(5)
    n_seg, n_bins, t = 9, 64, 16.0
    P = g.uniform(0.5, 2.0, (n_seg, n_bins)).astype(np.float32).astype(np.float64)
    f0 = g.uniform(0, n_bins, n_seg) / t
    U = g.standard_normal((n_seg, 2)) / t * 8
    C = g.uniform(-4, 4, (700, 2)).astype(np.float32)
    C[3] = [np.inf, 0.0]
    C[4] = [np.nan, 1.0]
    C[5] = [3e38, -3e38]
    C[6] = [1e9, 0.0]
    kmin, kmax = k_range
    kw = dict(k_min=kmin, k_max=-1 if kmax is None else kmax)
    gpu = score_gpu(gpu_lib, P, f0, U, C, t, 10, want_bins=True, want_near_tie=True, **kw)
    o = oracle.score_tracks(P, f0, U, C, t, 10, k_min=kmin, k_max=kmax, want_bins=True)
    check_against_oracle(P, f0, U, C, t, gpu, o, kmin, kmax)
    assert gpu["stat"][3] == 0 and gpu["stat"][4] == 0 and gpu["stat"][5] == 0 and gpu["stat"][6] == 0
    fast = score_gpu(gpu_lib, P, f0, U, C, t, 10, **kw)
    assert np.array_equal(fast["stat"], gpu["stat"])
    check_topk(fast["topk_val"], fast["topk_idx"], o["stat"], 10)


def test_column_sum_k0(gpu_lib):
    g = np.random.default_rng(31)
    n_seg, n_bins, t = 9, 100, 1000.0
    P = g.exponential(size=(n_seg, n_bins)).astype(np.float32).astype(np.float64)
    for b in (0, 1, 57, 99):
        f0 = np.full(n_seg, b / t)
        gpu = score_gpu(gpu_lib, P, f0, np.zeros((n_seg, 0)), np.zeros((1000, 0), np.float32), t, 5)
        assert np.allclose(gpu["stat"], P[:, b].sum(), rtol=1e-6, atol=0)
        assert np.all(gpu["stat"] == gpu["stat"][0])
        assert list(gpu["topk_idx"]) == [0, 1, 2, 3, 4]          # all tied: lowest indices


@pytest.mark.parametrize("K", [1, 3, 4, 5, 8, 12, 16, 32])
def test_ragged_sizes_and_K(gpu_lib, K):
    """Several tiles and a ragged tail for each compiled K."""
    g = np.random.default_rng(100 + K)
    n_seg, t = 37, 163840.0
    n_bins = 3001
    P = g.exponential(size=(n_seg, n_bins)).astype(np.float32).astype(np.float64)
    f0 = g.uniform(200, 2800, n_seg) / t
    U = np.linalg.qr(g.standard_normal((n_seg, K)))[0] * (30.0 / t)
    n = 3 * 4608 + 777 if K <= 8 else 2 * 2560 + 123
    C = g.uniform(-60, 60, (n, K)).astype(np.float32)
    gpu = score_gpu(gpu_lib, P, f0, U, C, t, 64, want_bins=True, want_near_tie=True)
    o = oracle.score_tracks(P, f0, U, C, t, 64, want_bins=True)
    check_against_oracle(P, f0, U, C, t, gpu, o)
    fast = score_gpu(gpu_lib, P, f0, U, C, t, 64)
    assert np.array_equal(fast["stat"], gpu["stat"])            # same arithmetic, same order
    check_topk(fast["topk_val"], fast["topk_idx"], o["stat"], 64)
    assert np.array_equal(fast["topk_val"], fast["stat"][fast["topk_idx"]])


def test_many_tiles_per_workgroup(gpu_lib):
    """Enough templates that every workgroup walks several full tiles and a partial one."""
    g = np.random.default_rng(9)
    n_seg, n_bins, t = 12, 2049, 40960.0
    P = g.exponential(size=(n_seg, n_bins)).astype(np.float32).astype(np.float64)
    f0 = g.uniform(300, 1700, n_seg) / t
    U = np.linalg.qr(g.standard_normal((n_seg, 8)))[0] * (40.0 / t)
    n = 2 * 256 * 4608 + 12345
    C = g.uniform(-30, 30, (n, 8)).astype(np.float32)
    gpu = score_gpu(gpu_lib, P, f0, U, C, t, 256)
    o = oracle.score_tracks(P, f0, U, C, t, 256)
    x_rows = np.nonzero(np.abs(gpu["stat"] - o["stat"]) > STAT_RTOL * np.abs(o["stat"]))[0]
    for j in x_rows:       # only near-tie templates may differ more, and then by a bin choice
        x = oracle.track_positions(f0, U, C[j:j + 1], t)
        assert oracle.near_tie_mask(x).any(), j
    check_topk(gpu["topk_val"], gpu["topk_idx"], o["stat"], 256)


def test_config0_parity_and_injection(gpu_lib):
    import torch
    emri = gpu_lib
    st = synth.stream_config0()
    P = oracle.build_sfts(st["x"], st["dt"], st["n_sft"], st["psd"])
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], st["K"])
    t = st["n_sft"] * st["dt"]
    C = synth.coefficients(0, 0, st["n_tmpl"], lo, hi)
    inj = st["injection"]
    c_true = (U.T @ (synth.chirp_frequency(st["t_mid"], inj["f0"], inj["tau"]) - f0)).astype(np.float32)
    C = np.vstack([C, c_true[None, :]])
    # GPU-built spectrogram, scored on the GPU
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]))
    res = emri.score_tracks(spec, _t(f0), _t(U), _t(C), st["top_k"], want_bins=True, want_near_tie=True)
    torch.cuda.synchronize()
    gpu = {k: _np(v) for k, v in res.items()}
    P_gpu = _np(spec.power()).astype(np.float64)
    o = oracle.score_tracks(P, f0, U, C, t, st["top_k"], want_bins=True)
    # bins depend only on the positions; statistics on P (GPU power vs oracle power)
    check_against_oracle(P, f0, U, C, t, gpu, o)
    check_topk(gpu["topk_val"], gpu["topk_idx"], o["stat"], st["top_k"])
    assert gpu["topk_idx"][0] == st["n_tmpl"]
    from scipy import stats
    assert gpu["stat"][-1] > stats.gamma(30).ppf(0.999)


def test_fp16_power(gpu_lib):
    st = synth.stream_config0()
    P = oracle.build_sfts(st["x"], st["dt"], st["n_sft"], st["psd"])
    P16 = P.astype(np.float16).astype(np.float64)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], st["K"])
    t = st["n_sft"] * st["dt"]
    C = synth.coefficients(0, 0, 3000, lo, hi)
    gpu = score_gpu(gpu_lib, P16, f0, U, C, t, 16, dtype="f16", want_bins=True, want_near_tie=True)
    o = oracle.score_tracks(P16, f0, U, C, t, 16, want_bins=True)
    check_against_oracle(P16, f0, U, C, t, gpu, o)
    fast = score_gpu(gpu_lib, P16, f0, U, C, t, 16, dtype="f16")
    assert np.array_equal(fast["stat"], gpu["stat"])
    check_topk(fast["topk_val"], fast["topk_idx"], o["stat"], 16)


def test_topk_ties_and_padding(gpu_lib):
    g = np.random.default_rng(77)
    n_seg, n_bins, t = 5, 50, 100.0
    P = np.round(g.exponential(size=(n_seg, n_bins)), 0)       # integers: many exact ties
    f0 = g.uniform(5, 45, n_seg) / t
    U = g.standard_normal((n_seg, 2)) * 0.05
    C = g.uniform(-1, 1, (20000, 2)).astype(np.float32)
    for k in (1, 7, 100, 1000, 4096):
        gpu = score_gpu(gpu_lib, P, f0, U, C, t, k)
        ov, oi = oracle.topk_order(gpu["stat"].astype(np.float64), k)
        assert np.array_equal(gpu["topk_idx"], oi), k          # exact order incl. index tie-break
        assert np.array_equal(gpu["topk_val"], ov.astype(np.float32))
    small = score_gpu(gpu_lib, P, f0, U, C[:3], t, 8)
    assert list(small["topk_idx"][3:]) == [-1] * 5 and np.all(np.isneginf(small["topk_val"][3:]))
    empty = score_gpu(gpu_lib, P, f0, U, C[:0], t, 4)
    assert list(empty["topk_idx"]) == [-1] * 4
    none = score_gpu(gpu_lib, P, f0, U, C[:100], t, 0)
    assert none["stat"].shape == (100,)


@pytest.mark.parametrize("n,k,rare", [(3_000_000, 4096, False), (3_000_000, 4096, True), (1_234_567, 777, True),
                                       (4097, 4096, False), (70_000, 1, True)])
def test_topk_massive_ties(gpu_lib, n, k, rare):
    """Three distinct statistic values over up to 3e6 templates: the k-th value is
    shared by far more templates than are needed, so the index passes decide
    (over two index digits at 3e6), and equal keys fill whole waves.  `rare`:
    the two larger values are rare, so the cut falls among the ties of the
    smallest value, below elements that are all taken."""
    n_seg, n_bins, t = 1, 64, 1.0
    P = np.ones((n_seg, n_bins))
    P[0, 3], P[0, 7] = 5.0, 4.0
    g = np.random.default_rng(n + k)
    if rare:
        c = np.where(g.random(n) < 5e-4, 3, np.where(g.random(n) < 5e-4, 7, g.integers(8, 64, n)))
    else:
        c = g.integers(0, 64, n)
    C = c.astype(np.float32)[:, None]                  # position = bin, exactly
    gpu = score_gpu(gpu_lib, P, np.zeros(n_seg), np.ones((n_seg, 1)), C, t, k)
    assert np.array_equal(gpu["stat"], P[0, c].astype(np.float32))
    ov, oi = oracle.topk_order(P[0, c], k)
    assert np.array_equal(gpu["topk_idx"], oi)
    assert np.array_equal(gpu["topk_val"], ov.astype(np.float32))


@pytest.mark.parametrize("sigma,k", [(3.0, 256), (0.05, 4096), (0.05, 1000)])
def test_topk_of_wide_and_narrow_statistics(gpu_lib, sigma, k):
    """2e6 templates whose statistics span many binades (lognormal sigma 3: the
    leading key digit takes many values) or one (sigma 0.05: a few values of the
    leading digit hold everything).  The selection must be exactly the first k
    of the statistic the GPU returned, ordered by (-S, index)."""
    g = np.random.default_rng(int(sigma * 100) + k)
    n_seg, n_bins, t, n = 3, 4096, 1.0, 2_000_000
    P = np.exp(g.normal(0.0, sigma, (n_seg, n_bins)))
    if sigma > 1:
        P[:, ::7] *= -1.0                                # negative values too
    f0 = np.array([100.0, 900.0, 2000.0])
    U = g.uniform(-1.0, 1.0, (n_seg, 2)) * 400.0
    C = g.uniform(-2.0, 2.0, (n, 2)).astype(np.float32)
    gpu = score_gpu(gpu_lib, P, f0, U, C, t, k)
    ov, oi = oracle.topk_order(gpu["stat"].astype(np.float64), k)
    assert np.array_equal(gpu["topk_idx"], oi)
    assert np.array_equal(gpu["topk_val"], ov.astype(np.float32))


@pytest.mark.parametrize("n_close,k", [(1500, 256), (1900, 256), (300, 1000), (5, 2000)])
def test_topk_boundary_sizes(gpu_lib, n_close, k):
    """n_close templates land on bins whose power differs only in the lowest
    mantissa bits (their keys share the 22 leading bits, with repeats), the
    rest on bins of power 0.5.  Depending on n_close + k the last key pass
    either gathers the boundary keys (up to 2048 words) or falls back to the
    radix passes; both must give exactly the first k by (-S, index)."""
    n, n_bins, t = 200_000, 2048, 1.0
    P = np.full((1, n_bins), 0.5)
    P[0, :1024] = 1.0 + np.arange(1024) * 2.0 ** -23
    g = np.random.default_rng(n_close + k)
    c = g.integers(1024, 2048, n)
    close = g.choice(n, n_close, replace=False)
    c[close] = g.integers(0, 1024, n_close)
    gpu = score_gpu(gpu_lib, P, np.zeros(1), np.ones((1, 1)), c.astype(np.float32)[:, None], t, k)
    assert np.array_equal(gpu["stat"], P[0, c].astype(np.float32))
    ov, oi = oracle.topk_order(P[0, c], k)
    assert np.array_equal(gpu["topk_idx"], oi)
    assert np.array_equal(gpu["topk_val"], ov.astype(np.float32))


def test_topk_nan_and_negative(gpu_lib):
    n_seg, n_bins, t = 2, 8, 1.0
    P = np.array([[1, -3, np.nan, 0, 2, 5, -0.0, 4], [0, 0, 0, 0, 0, 0, 0, 0]], dtype=np.float64)
    f0 = np.zeros(n_seg)
    U = np.ones((n_seg, 1))
    C = np.array([[0], [1], [2], [3], [4], [5], [6], [7], [2], [1]], dtype=np.float32)
    gpu = score_gpu(gpu_lib, P, f0, U, C, t, 10)
    # NaN ranks last; -0 equals +0 (index order between 3 and 6)
    assert list(gpu["topk_idx"]) == [5, 7, 4, 0, 3, 6, 1, 9, 2, 8]


def _sampled(n):
    """Templates the sampled threshold reads: one unit of 64 in every 16 (the
    statistics past the last whole group of 4 are never sampled)."""
    i = np.arange(n)
    return ((i // 64) % 16 == 0) & (i < 4 * (n // 4))


@pytest.mark.parametrize("case,k", [("spread", 1), ("spread", 100), ("spread", 256), ("sample_high", 256),
                                    ("sample_high", 7), ("one_value", 32), ("spread", 257)])
def test_topk_sampled_threshold(gpu_lib, case, k):
    """Top-k of 2^16 + 4099 statistics through the validating launch, which
    does not fuse the first key pass, so that k <= 256 takes the sampled
    threshold.  `spread`: 8192 distinct values, each held by ~128 templates in
    random order (the gathered candidates contain the top-k); `sample_high`:
    every sampled template scores above every other, so at k = 256 fewer than
    k are gathered and the radix passes decide; `one_value`: all equal, far
    more than 2048 are gathered and the radix passes decide by index; k = 257
    never samples.  Each must be exactly the first k by (-S, index)."""
    n, n_bins, t = (1 << 16) + 4099, 8192, 1.0
    g = np.random.default_rng(k + 10 * len(case))
    P = np.sort(g.uniform(1.0, 2.0, (1, n_bins))).astype(np.float32).astype(np.float64)
    if case == "one_value":
        P[:] = 1.5
    c = g.integers(0, n_bins, n)
    if case == "sample_high":
        c = np.where(_sampled(n), g.integers(n_bins // 2, n_bins, n), g.integers(0, n_bins // 2, n))
    gpu = score_gpu(gpu_lib, P, np.zeros(1), np.ones((1, 1)), c.astype(np.float32)[:, None], t, k,
                    want_near_tie=True)
    assert np.array_equal(gpu["stat"], P[0, c].astype(np.float32))
    ov, oi = oracle.topk_order(P[0, c], k)
    assert np.array_equal(gpu["topk_idx"], oi)
    assert np.array_equal(gpu["topk_val"], ov.astype(np.float32))


def test_one_year_full_size_sampled(gpu_lib):
    """1e7 templates at K = 8 on the one-year stream, in the launch the benchmark
    times: 2e4 sampled templates (plus the top-k and both ends) against the
    oracle, with near-ties judged at the GPU's own bins (the validation kernel
    re-scores the sampled rows with the same arithmetic and summation order and
    must reproduce the full launch's statistics bit for bit); and the top-256
    against the oracle's exact top-256 over every template whose GPU statistic
    could reach it (all within 3e-5 of the GPU's 256th value, which contains the
    oracle's top-256 because every statistic is within 1e-5 of the oracle's)."""
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], st["K"])
    n, k = st["n_tmpl"], st["top_k"]
    C = synth.coefficients(1, 0, n, lo, hi)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]))
    f0_d, U_d, C_d = _t(f0), _t(U), _t(C)
    res = emri.score_tracks(spec, f0_d, U_d, C_d, k)
    torch.cuda.synchronize()
    stat = _np(res["stat"])
    top_idx, top_val = _np(res["topk_idx"]), _np(res["topk_val"])
    P_gpu = _np(spec.power()).astype(np.float64)
    t = spec.t_sft
    assert np.array_equal(top_val, stat[top_idx])

    def rescore(rows):
        val = emri.score_tracks(spec, f0_d, U_d, _t(C[rows]), 0, want_bins=True, want_near_tie=True)
        torch.cuda.synchronize()
        val = {key: _np(v) for key, v in val.items()}
        assert np.array_equal(val["stat"], stat[rows])
        o = oracle.score_tracks(P_gpu, f0, U, C[rows], t, 0, want_bins=True)
        check_against_oracle(P_gpu, f0, U, C[rows], t, val, o)
        return oracle.score.fsum_rows(P_gpu, val["bins"].astype(np.int64))

    g = np.random.default_rng(1)
    rescore(np.unique(np.concatenate([g.integers(0, n, 20000), top_idx, [0, n - 1]])))
    kth = float(top_val[k - 1])
    cand = np.flatnonzero(stat >= kth - 3e-5 * abs(kth))
    assert k <= cand.size < 200_000, cand.size
    ref = np.full(n, -np.inf)
    ref[cand] = rescore(cand)
    check_topk(top_val, top_idx, ref, k)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("n_seg,n_bins,pitch,k_range", [
    (7, 256, 256, (0, None)),       # no padding: one row per step; rows of exactly 1 KB (f32)
    (9, 256, 264, (0, None)),       # padded: several rows per step, ragged final step
    (5, 513, 520, (3, 500)),        # bin range inside the row
    (13, 1000, 1000, (1, 998)),     # no padding, interior range
    (11, 4321, 4328, (0, None)),    # config-0 row length
])
def test_staging_geometries_with_dirty_padding(gpu_lib, dtype, n_seg, n_bins, pitch, k_range):
    """Row padding holds huge values that must never be gathered; fast and validation kernels
    agree bit for bit, and both match the oracle."""
    import torch
    emri = gpu_lib
    g = np.random.default_rng(n_bins + pitch)
    t = 1000.0
    P = g.exponential(size=(n_seg, n_bins))
    data = np.full((n_seg, pitch), 3.0e4)
    data[:, :n_bins] = P
    tdtype = torch.float32 if dtype == "f32" else torch.float16
    spec = emri.Spectrogram(_t(data).to(tdtype), n_bins, t)
    P_used = _np(spec.power()).astype(np.float64)
    K = 3
    f0 = g.uniform(0.1, 0.9, n_seg) * n_bins / t
    U = g.standard_normal((n_seg, K)) * (n_bins / 6 / t)
    C = g.uniform(-1.5, 1.5, (3000, K)).astype(np.float32)
    k_min, k_max = k_range[0], (n_bins - 1 if k_range[1] is None else k_range[1])
    args = (spec, _t(f0), _t(U), _t(C), 16)
    fast = emri.score_tracks(*args, k_min=k_min, k_max=k_max)
    val = emri.score_tracks(*args, k_min=k_min, k_max=k_max, want_bins=True, want_near_tie=True)
    torch.cuda.synchronize()
    fast, val = ({k: _np(v) for k, v in r.items()} for r in (fast, val))
    assert np.array_equal(fast["stat"], val["stat"])
    o = oracle.score_tracks(P_used, f0, U, C, t, 16, k_min, k_max, want_bins=True)
    check_against_oracle(P_used, f0, U, C, t, val, o, k_min, k_max)
    assert fast["stat"].max() < 3.0e4 * 0.5


def test_two_streams_in_flight_match_standalone(gpu_lib):
    """Two calls queued on two streams at once, each with the binding's default
    workspace for its stream: both results equal the same calls made alone."""
    import torch
    emri = gpu_lib
    g = np.random.default_rng(77)
    cases = []
    for n_seg, n_bins, n in ((40, 3000, 300_000), (25, 5000, 200_000)):
        t = 2000.0
        P = g.exponential(size=(n_seg, n_bins))
        spec = emri.spectrogram_from_power(P, t, "f32")
        f0 = g.uniform(0.3, 0.7, n_seg) * n_bins / t
        U = g.standard_normal((n_seg, 8)) * (40.0 / t)
        C = g.uniform(-3, 3, (n, 8)).astype(np.float32)
        cases.append((spec, _t(f0), _t(U), _t(C)))
    alone = []
    for spec, f0, U, C in cases:
        r = emri.score_tracks(spec, f0, U, C, 64)
        torch.cuda.synchronize()
        alone.append({k: v.clone() for k, v in r.items()})
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    outs = []
    for rep in range(3):
        outs = [emri.score_tracks(*cases[i], 64, stream=streams[i]) for i in range(2)]
    torch.cuda.synchronize()
    for got, ref in zip(outs, alone):
        for key in ("stat", "topk_val", "topk_idx"):
            assert torch.equal(got[key], ref[key]), key
