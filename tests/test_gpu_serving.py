"""Serving form on the GPU: requests arriving while others run are batched
continuously across several resident spectrograms, and every request's top-k
is bit for bit the result of a standalone score_tracks call."""
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
