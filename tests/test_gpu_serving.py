"""Serving form on the GPU: requests arriving while others run are batched
continuously across several resident spectrograms; every request's top-k is
bit for bit the result of a standalone score_tracks call, and every request is
checked against the FP64 oracle on its own spectrogram."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_serving_results_equal_standalone(gpu_lib, precision):
    import torch
    emri = gpu_lib
    from paper_2510_20891_amd.serving import GpuExecutor, Request, Server
    g = np.random.default_rng(42)
    K, t = 8, 3000.0
    specs, f0s, Us, segs = [], [], [], []
    for s, (n_seg, n_bins) in enumerate([(24, 2000), (40, 3500), (9, 700)]):
        P = g.exponential(size=(n_seg, n_bins))
        specs.append(emri.spectrogram_from_power(P, t, "f16"))
        f0s.append(torch.from_numpy(g.uniform(0.3, 0.7, n_seg) * n_bins / t).cuda())
        Us.append(torch.from_numpy(g.standard_normal((n_seg, K)) * (25.0 / t)).cuda())
        segs.append(n_seg)
    reqs = []
    tt = 0.0
    for i in range(240):
        tt += g.exponential(1 / 3000.0)
        n = int(np.exp(g.uniform(np.log(16), np.log(6000))))
        reqs.append(Request(i, int(g.integers(0, 3)), g.uniform(-4, 4, (n, K)).astype(np.float32),
                            int(g.integers(1, 33)), tt))
    ex = GpuExecutor(specs, f0s, Us, K, slots=3, max_batch_templates=40000, max_requests=64, top_k=32,
                     precision=precision)
    srv = Server(ex, K, hbm_budget=4 << 20, max_batch_templates=40000, max_requests=64, slots=3, seg_counts=segs)
    srv.run(reqs)
    assert len(srv.done) == len(reqs)
    assert srv.batches < len(reqs)                  # requests were batched together
    for r in reqs:
        ref = emri.score_tracks(specs[r.stream], f0s[r.stream], Us[r.stream], torch.from_numpy(r.coeffs).cuda(),
                                r.top_k, precision=precision)
        torch.cuda.synchronize()
        assert np.array_equal(ref["topk_idx"].cpu().numpy(), r.topk_idx), r.rid
        assert np.array_equal(ref["topk_val"].cpu().numpy(), r.topk_val), r.rid
    st = srv.stats(reqs)
    assert st.latency_ms["p50"] > 0 and st.n_requests == len(reqs)
    check_served_against_oracle(emri, specs, f0s, Us, reqs, precision)


def check_served_against_oracle(emri, specs, f0s, Us, reqs, precision):
    """Every served top-k against the FP64 oracle on the request's own spectrogram.

    Plain: the top-k equals the oracle's exact top-k of the request's batch (as
    a set, up to entries within 2e-5 of the k-th value), with near-tie positions
    judged at the GPU's bins (from a standalone validation call, whose
    statistic the served values must equal).  Mixed: the served values are
    within 2e-3 of the oracle's statistic of the same templates at p99, and the
    served top-k sets hold at least 99 % of the oracle's top-k entries."""
    import torch
    import oracle
    from tests.test_gpu_parity import check_topk
    rel_all, hit, want = [], 0, 0
    for r in reqs:
        P = specs[r.stream].power().cpu().numpy().astype(np.float64)
        f0 = f0s[r.stream].cpu().numpy()
        U = Us[r.stream].cpu().numpy()
        o = oracle.score_tracks(P, f0, U, r.coeffs, specs[r.stream].t_sft, r.top_k, want_bins=True)
        if precision == "plain":
            val = emri.score_tracks(specs[r.stream], f0s[r.stream], Us[r.stream], torch.from_numpy(r.coeffs).cuda(),
                                    0, want_bins=True, want_near_tie=True)
            torch.cuda.synchronize()
            gb = val["bins"].cpu().numpy().astype(np.int64)
            near = oracle.near_tie_mask(oracle.track_positions(f0, U, r.coeffs, specs[r.stream].t_sft))
            assert np.all((gb == o["bins"]) | near), r.rid
            ref = oracle.score.fsum_rows(P, gb)
            live = r.topk_idx >= 0
            assert np.array_equal(val["stat"].cpu().numpy()[r.topk_idx[live]], r.topk_val[live]), r.rid
            check_topk(r.topk_val, r.topk_idx, ref, r.top_k)
        else:
            live = r.topk_idx[r.topk_idx >= 0]
            assert live.size == min(r.top_k, r.n), r.rid
            rel_all.append(np.abs(r.topk_val[: live.size] - o["stat"][live]) / np.abs(o["stat"][live]))
            hit += len(set(live.tolist()) & set(o["topk_idx"][: live.size].tolist()))
            want += live.size
    if precision != "plain":
        rel = np.concatenate(rel_all)
        assert np.quantile(rel, 0.99) <= 2e-3, np.quantile(rel, 0.99)
        assert hit >= 0.99 * want, (hit, want)
