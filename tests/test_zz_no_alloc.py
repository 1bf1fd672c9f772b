"""score_tracks_noalloc (static scratch, no allocation) against score_tracks
through the C ABI: two calls in a row on one GPU, the second smaller, both
equal to the workspace entry point's results bit for bit; a request too
large for the scratch is refused and leaves the next call unaffected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(emri, g, n_seg, n_bins, n, K, dtype):
    import torch
    t = 1500.0
    P = g.exponential(size=(n_seg, n_bins))
    spec = emri.spectrogram_from_power(P, t, dtype)
    f0 = torch.from_numpy(g.uniform(0.3, 0.7, n_seg) * n_bins / t).cuda()
    U = torch.from_numpy(g.standard_normal((n_seg, K)) * (30.0 / t)).cuda()
    C = torch.from_numpy(g.uniform(-3, 3, (n, K)).astype(np.float32)).cuda()
    return spec, f0, U, C


@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_noalloc_equals_workspace_entry_point(gpu_lib, precision):
    import torch
    emri = gpu_lib
    g = np.random.default_rng(2024)
    dtype = "f16" if precision == "mixed" else "f32"
    for n_seg, n_bins, n, K, top_k in ((192, 8193, 400_000, 8, 256), (37, 3001, 20_000, 8, 40)):
        spec, f0, U, C = _case(emri, g, n_seg, n_bins, n, K, dtype)
        ref = emri.score_tracks(spec, f0, U, C, top_k, precision=precision)
        torch.cuda.synchronize()
        stat = torch.full((n,), -7.0, dtype=torch.float32, device="cuda")
        val = torch.empty(top_k, dtype=torch.float32, device="cuda")
        idx = torch.empty(top_k, dtype=torch.int64, device="cuda")
        emri.score_tracks_noalloc(spec, f0, U, C, top_k, stat, val, idx, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(stat, ref["stat"])
        assert torch.equal(val, ref["topk_val"])
        assert torch.equal(idx, ref["topk_idx"])
    # without a statistic output the statistic lives in the scratch; too many templates are refused
    spec, f0, U, C = _case(emri, g, 12, 900, 5000, 4, dtype)
    big = torch.zeros((2_000_000, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(emri.EmriError) as err:
        emri.score_tracks_noalloc(spec, f0, U, big, 8, None, torch.empty(8, device="cuda"),
                                  torch.empty(8, dtype=torch.int64, device="cuda"), precision=precision)
    assert err.value.status == -3
    ref = emri.score_tracks(spec, f0, U, C, 8, precision=precision)
    val = torch.empty(8, dtype=torch.float32, device="cuda")
    idx = torch.empty(8, dtype=torch.int64, device="cuda")
    emri.score_tracks_noalloc(spec, f0, U, C, 8, None, val, idx, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(val, ref["topk_val"]) and torch.equal(idx, ref["topk_idx"])
