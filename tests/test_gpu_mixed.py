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
@pytest.mark.parametrize("n_seg,n_tmpl", [(n, 7000) for n in (1, 2, 3, 5, 6, 7, 8, 9, 10, 11, 12)] +
                         [(n, 1_600_000) for n in (1, 3, 5, 8, 11)])
def test_mixed_short_and_ragged_segment_counts(gpu_lib, K, n_seg, n_tmpl):
    """Every position of the last staging step (4 segments) and of the last
    loop turn (two steps); up to K = 8 the kernel keeps the gathers of two
    segments in flight, at K = 16 one.  With 7000 templates the 14 workgroups
    get 500 templates each, so only the half-size tail tile runs (with idle
    lanes); with 1.6e6 templates each of the (up to 256) workgroups gets about
    6250, so full tiles of TPL x 768 or x 1024 templates (2304 to 4096) run before a
    ragged tail."""
    emri = gpu_lib
    g = np.random.default_rng(1000 + 17 * K + n_seg + n_tmpl)
    n_bins, t = 600, 1.0
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, "f16")
    f0 = np.round(g.uniform(200, 400, n_seg)) + 0.25
    U = g.integers(-3, 4, (n_seg, K)).astype(np.float64)
    C = (g.integers(-16, 17, (n_tmpl, K)) / 2.0).astype(np.float32)
    plain = _score(emri, spec, f0, U, C, 16)
    mixed = _score(emri, spec, f0, U, C, 16, precision="mixed")
    assert np.array_equal(plain["stat"], mixed["stat"])
    assert np.array_equal(plain["topk_idx"], mixed["topk_idx"])
    rows = np.arange(n_tmpl) if n_tmpl <= 10000 else np.unique(np.r_[np.arange(0, n_tmpl, 331), n_tmpl - 1])
    o = oracle.score_tracks(_np(spec.power()).astype(np.float64), f0, U, C[rows], t, 0)
    assert np.max(np.abs(mixed["stat"][rows] - o["stat"]) / np.maximum(o["stat"], 1e-30)) <= 1e-5


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


@pytest.mark.parametrize("K", [8, 16])
def test_mixed_one_year_full_size_error_report(gpu_lib, K):
    """The one-year stream at its full shape (1e7 templates uniform in the K-basis
    box, FP16 power): the statistic error against the FP64 oracle (on the same
    FP16 power) on 3e4 sampled templates, p99 <= 2e-3 with the maximum bounded
    by one flipped bin (the FP32 accumulation can move a position that lies
    within ~1e-3 bin of a half-integer to the neighbouring bin); and the top-100
    overlap with the oracle's exact top-100, found by scoring with the oracle
    the union of the plain and mixed top-2000 (the plain statistic is within
    1e-5 of the oracle's, so that union holds the oracle's top-100)."""
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], K)
    n = st["n_tmpl"]
    C = synth.coefficients(1, K, n, lo, hi)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="f16")
    C_d = _t(C)
    res = emri.score_tracks(spec, _t(f0), _t(U), C_d, 100, precision="mixed")
    plain = emri.score_tracks(spec, _t(f0), _t(U), C_d, 100)
    torch.cuda.synchronize()
    stat = _np(res["stat"])
    P16 = _np(spec.power()).astype(np.float64)
    rows = np.random.default_rng(3 + K).integers(0, n, 30000)
    o = oracle.score_tracks(P16, f0, U, C[rows], spec.t_sft, 0)
    rel = np.abs(stat[rows] - o["stat"]) / np.abs(o["stat"])
    q = np.quantile(rel, [0.5, 0.99, 1.0])
    print(f"mixed K={K}: statistic relative error p50 {q[0]:.2e} p99 {q[1]:.2e} max {q[2]:.2e}")
    assert q[1] <= 2e-3, q
    assert q[2] <= 0.1, q
    cand = np.unique(np.concatenate([_np(torch.topk(res["stat"], 2000).indices),
                                     _np(torch.topk(plain["stat"], 2000).indices)]))
    oc = oracle.score_tracks(P16, f0, U, C[cand], spec.t_sft, 100)
    true_top = set(cand[oc["topk_idx"]].tolist())
    overlap = len(true_top & set(_np(res["topk_idx"]).tolist()))
    print(f"mixed K={K}: top-100 overlap {overlap}")
    assert overlap >= 99
    assert np.array_equal(_np(res["topk_val"]), stat[_np(res["topk_idx"])])
    # re-scoring the leading candidates returns the oracle's top-100
    resc = emri.score_tracks(spec, _t(f0), _t(U), C_d, 100, precision="mixed", rescore_top=True)
    torch.cuda.synchronize()
    ridx = _np(resc["topk_idx"])
    assert set(ridx.tolist()) == true_top
    assert np.array_equal(ridx, _np(plain["topk_idx"]))


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


@pytest.mark.parametrize("n_seg,n_bins,n_tmpl,K,top_k,dtype", [
    (23, 700, 5000, 8, 32, "f16"),
    (600, 300, 3000, 3, 16, "f32"),        # more than one chunk of 512 segments, a ragged last run
    (9, 500, 50, 16, 16, "f16"),           # fewer templates than candidates
    (9, 500, 10, 4, 16, "f16"),            # top_k larger than the batch: padded
    (40, 4000, 200_000, 8, 100, "f16"),    # general inputs, many moved bins in the mixed statistic
])
def test_mixed_rescore_top_matches_plain(gpu_lib, n_seg, n_bins, n_tmpl, K, top_k, dtype):
    """rescore_top: the returned top-k is the plain path's top-k, values bit for
    bit, and the re-scored entries of stat are the plain statistic."""
    emri = gpu_lib
    g = np.random.default_rng(400 + n_seg + K)
    t = 1.0
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, dtype)
    f0 = g.uniform(0.4 * n_bins, 0.6 * n_bins, n_seg)
    U = g.standard_normal((n_seg, K)) * (0.02 * n_bins)
    C = g.uniform(-2, 2, (n_tmpl, K)).astype(np.float32)
    plain = _score(emri, spec, f0, U, C, top_k)
    mixed = _score(emri, spec, f0, U, C, top_k, precision="mixed")
    resc = _score(emri, spec, f0, U, C, top_k, precision="mixed", rescore_top=True)
    kk = min(top_k, n_tmpl)
    assert np.array_equal(resc["topk_idx"][:kk], plain["topk_idx"][:kk])
    assert np.array_equal(resc["topk_val"][:kk], plain["topk_val"][:kk])
    assert np.all(resc["topk_idx"][kk:] == -1) and np.all(np.isneginf(resc["topk_val"][kk:]))
    assert np.array_equal(resc["stat"][resc["topk_idx"][:kk]], plain["stat"][resc["topk_idx"][:kk]])
    # entries that were not re-scored keep the mixed statistic
    changed = np.flatnonzero(resc["stat"] != mixed["stat"])
    n_cand = min(n_tmpl, max(4 * top_k, 64), 4096)
    assert changed.size <= n_cand
    assert np.array_equal(resc["stat"][changed], plain["stat"][changed])
    # and the top-k agrees with the oracle's on its own candidates
    o = oracle.score_tracks(_np(spec.power()).astype(np.float64), f0, U, C[resc["topk_idx"][:kk]], t, 0)
    assert np.max(np.abs(resc["topk_val"][:kk] - o["stat"]) / np.maximum(o["stat"], 1e-30)) <= 1e-5


@pytest.mark.parametrize("case,K", [("few_queued", 16), ("few_queued", 13), ("few_queued", 12),
                                    ("few_queued", 9), ("all_queued", 16), ("all_queued", 12),
                                    ("queue_overflow", 16)])
def test_mixed_reduced_chain_queue(gpu_lib, case, K):
    """Above K = 8 the mixed form runs the reduced chain (order <= 1 products
    for coefficients 8..11, the leading product alone for 12..15) and queues,
    per wave, the tiles holding a template whose last two coefficient groups
    are not small enough for it; the full chains then score the queued tiles
    again (or everything once the queue overflows), writing only the
    templates that need them.  So each statistic depends on its own template
    only, and the batched form (the same launches over work items) equals
    standalone calls bit for bit, as does a call on a slice of the batch
    (other tiles).  In "few_queued" the basis decays (groups 2 and 3 scaled
    by 1e-4 and 1e-7) and a handful of templates carry group-3 terms of up to
    ~450 bins per coefficient (K > 12; left-out products of order 1 move
    positions by whole bins) or group-2 terms of up to ~225 bins (K <= 12;
    left-out products of order 2 move them by a few hundredths): those
    templates must match the FP64 oracle to 1e-6 wherever no position lies
    within 1e-3 bin of a half-integer.  "all_queued" and "queue_overflow" use a basis that does
    not decay, so every wave queues (about 520 and 3100 queue entries
    against a capacity of 1024).  K = 13 has a single coefficient in group 3,
    K = 9 a single one in group 2."""
    import torch
    emri = gpu_lib
    g = np.random.default_rng({"few_queued": 81, "all_queued": 82, "queue_overflow": 83}[case] + K)
    n_seg, n_bins, t = {"few_queued": (40, 6000, 163840.0), "all_queued": (12, 3000, 163840.0),
                        "queue_overflow": (9, 3000, 163840.0)}[case]
    n = {"few_queued": 60000, "all_queued": 100000, "queue_overflow": 600000}[case]
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, "f16")
    f0 = g.uniform(0.45, 0.55, n_seg) * n_bins / t
    U = g.standard_normal((n_seg, K)) * (15.0 / t)
    C = g.uniform(-3, 3, (n, K)).astype(np.float32)
    if case == "few_queued":
        U[:, 8:12] *= 1e-4
        U[:, 12:] *= 1e-7
        bad = np.array([0, 5, 2303, 2304, 31000, 45678, n - 1])
        if K > 12:
            C[bad, 12:] = g.uniform(-1e8, 1e8, (bad.size, K - 12)).astype(np.float32)
        else:
            C[bad, 8:] = g.uniform(-5e4, 5e4, (bad.size, K - 8)).astype(np.float32)
    pb = emri.Problem(spec, _t(f0), _t(U), _t(C), top_k=50)
    emri.BatchPlan([pb], K, precision="mixed").run()
    torch.cuda.synchronize()
    got = _score(emri, spec, f0, U, C, 50, precision="mixed")
    assert np.array_equal(got["stat"], _np(pb.stat))
    assert np.array_equal(got["topk_idx"], _np(pb.topk_idx))
    if case == "few_queued":
        P_used = spec.power().cpu().numpy().astype(np.float64)
        # the planted templates took the full chains
        x = oracle.track_positions(f0, U, C[bad], spec.t_sft)
        clear = ~np.any(np.abs(np.abs(x - np.floor(x)) - 0.5) < 1e-3, axis=1)
        assert clear.sum() >= 3
        ob = oracle.score_tracks(P_used, f0, U, C[bad], spec.t_sft, 0)["stat"]
        assert np.all(np.abs(got["stat"][bad] - ob)[clear] <= 1e-6 * np.abs(ob)[clear])
        # the others ran the reduced chain: within the mixed form's tolerance
        rows = np.arange(0, n, 211)
        o = oracle.score_tracks(P_used, f0, U, C[rows], spec.t_sft, 0)
        rel = np.abs(got["stat"][rows] - o["stat"]) / np.abs(o["stat"])
        assert np.quantile(rel, 0.99) <= 2e-3
        sub = _score(emri, spec, f0, U, C[1000:], 0, precision="mixed")
        assert np.array_equal(sub["stat"], got["stat"][1000:])
