"""The C ABI on the CPU: the library loads, exports every declared symbol, and
rejects invalid arguments before touching the GPU.  build_basis is host code
and is checked against the oracle here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2510_20891_amd as emri
from paper_2510_20891_amd import _Opts, _Power

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "emri.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = emri.load()
    names = declared_functions()
    assert {"build_sfts", "build_basis", "score_tracks", "score_tracks_workspace_size",
            "emri_status_string", "emri_last_error"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(emri.SIGNATURES)


def test_status_strings():
    lib = emri.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.emri_status_string(code)
    assert b"unknown" in lib.emri_status_string(7)


def _power(n_seg=4, n_bins=33, pitch=40, dtype=0, t=100.0, data=0x1000):
    return _Power(data, n_seg, n_bins, pitch, dtype, t)


FAKE = 0x100000   # never dereferenced: validation fails first


def _score(pw, K=2, n=10, top_k=4, opts=None, ws_bytes=1 << 20, coeffs=FAKE, ws=FAKE, f0=FAKE, U=FAKE,
           vals=FAKE, idx=FAKE):
    lib = emri.load()
    return lib.score_tracks(ctypes.byref(pw), f0, U, K, coeffs, n, top_k, FAKE, vals, idx, None, None,
                            ctypes.byref(opts) if opts else None, ws, ws_bytes, None)


@pytest.mark.parametrize("case,status", [
    (dict(K=33), -1), (dict(K=-1), -1), (dict(n=-1), -1), (dict(top_k=4097), -1), (dict(top_k=-2), -1),
    (dict(coeffs=None), -1), (dict(ws=None), -1), (dict(vals=None), -1), (dict(f0=None), -1),
    (dict(coeffs=FAKE + 4), -1), (dict(ws=FAKE + 16), -1), (dict(ws_bytes=64), -3),
])
def test_score_tracks_rejects(case, status):
    assert _score(_power(), **case) == status
    assert emri.load().emri_last_error()


@pytest.mark.parametrize("pw,status", [
    (_power(pitch=36), -1), (_power(pitch=32), -1), (_power(n_bins=0), -1), (_power(dtype=3), -1),
    (_power(t=0.0), -1), (_power(t=float("inf")), -1), (_power(data=0), -1), (_power(n_seg=-1), -1),
    (_power(n_bins=30000, pitch=30000), -5),
])
def test_score_tracks_rejects_power(pw, status):
    assert _score(pw) == status


def test_score_tracks_rejects_bin_range():
    assert _score(_power(), opts=_Opts(5, 2)) == -1
    assert _score(_power(), opts=_Opts(-1, 3)) == -1
    assert _score(_power(), opts=_Opts(0, 33)) == -1
    bad = _Opts(0, -1)
    bad.reserved[2] = 1
    assert _score(_power(), opts=bad) == -1
    bad = _Opts(0, -1, 1)
    bad.rescore_top = 2
    assert _score(_power(), opts=bad) == -1


def test_workspace_size_grows_with_stat_in_workspace():
    lib = emri.load()
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    pw = _power()
    assert lib.score_tracks_workspace_size(ctypes.byref(pw), 8, 1000, 16, 0, ctypes.byref(a)) == 0
    assert lib.score_tracks_workspace_size(ctypes.byref(pw), 8, 1000, 16, 1, ctypes.byref(b)) == 0
    assert b.value >= a.value + 4000 and a.value % 256 == 0
    assert lib.score_tracks_workspace_size(ctypes.byref(pw), 8, 1000, 16, 1, None) == -1


def test_build_sfts_rejects():
    lib = emri.load()
    pw = _Power(FAKE, 0, 0, 8, 0, 0.0)
    call = lambda n_sft, dt=1.0, n=1000, pitch=8, x=FAKE, psd=FAKE, dtype=0: lib.build_sfts(
        x, n, dt, n_sft, psd, ctypes.byref(_Power(FAKE, 0, 0, pitch, dtype, 0.0)), None)
    assert call(7) == -1                  # odd
    assert call(2) == -1                  # too short
    assert call(16, dt=0.0) == -1
    assert call(16, dt=float("nan")) == -1
    assert call(16, pitch=4) == -1        # pitch < n_bins
    assert call(16, pitch=12) == -1       # pitch not a multiple of 8
    assert call(16, x=None) == -1
    assert call(16, x=FAKE + 8) == -1     # misaligned
    assert call(16, dtype=2) == -1
    assert call(22, pitch=16) == -5       # n_sft/2 = 11: prime factor above 7
    assert call(40960, pitch=20488) == -5  # beyond the LDS-resident FFT size
    assert lib.build_sfts(FAKE, 10, 1.0, 16, FAKE, None, None) == -1


def test_build_basis_rejects():
    lib = emri.load()
    F = np.ones((4, 3))
    out = np.empty(16)
    p = out.ctypes.data
    assert lib.build_basis(F.ctypes.data, 4, 3, 4, p, p, p, p, p) == -1       # K > n_seg
    assert lib.build_basis(None, 4, 3, 1, p, p, p, p, p) == -1
    F[1, 1] = np.nan
    assert lib.build_basis(F.ctypes.data, 4, 3, 1, p, p, p, p, p) == -1


def _chirps(n, n_seg, seed, t_sft):
    g = np.random.default_rng(seed)
    t = (np.arange(n_seg) + 0.5) * t_sft
    f0 = g.uniform(1e-3, 2e-2, n)
    tau = g.uniform(1, 10, n) * 3.15576e7
    return f0[:, None] * (1 - t[None, :] / tau[:, None]) ** -0.375


@pytest.mark.parametrize("n,n_seg,K", [(1000, 30, 4), (5000, 192, 8), (5000, 192, 16), (20, 40, 12)])
def test_build_basis_matches_oracle(n, n_seg, K):
    F = _chirps(n, n_seg, 7, 163840.0 if n_seg == 192 else 86400.0)
    f0, U, sv, lo, hi = emri.build_basis(F, K)
    of0, oU, osv, olo, ohi = oracle.build_basis(F, K)
    assert np.allclose(f0, of0, rtol=1e-14, atol=0)
    assert np.allclose(sv, osv, rtol=1e-9, atol=1e-12 * osv[0])
    assert np.abs(U.T @ U - np.eye(K)).max() < 1e-12
    for k in range(K):
        if osv[k] / osv[0] > 1e-6 and (k + 1 == K or osv[k + 1] < osv[k] * (1 - 1e-6)):
            assert np.abs(U[:, k] - oU[:, k]).max() < 1e-7, k          # same vector, same sign
            assert abs(lo[k] - olo[k]) <= 1e-6 * (ohi[k] - olo[k])
            assert abs(hi[k] - ohi[k]) <= 1e-6 * (ohi[k] - olo[k])
    # the kept subspace is the same (principal angles)
    cos = np.linalg.svd(U.T @ oU, compute_uv=False)
    keep = osv / osv[0] > 1e-6
    assert np.all(cos[: int(keep.sum())] > 1 - 1e-9)


def test_build_basis_full_rank_and_k0():
    F = _chirps(50, 10, 3, 86400.0)
    f0, U, sv, lo, hi = emri.build_basis(F, 10)
    X = F - f0
    assert np.abs(X @ U @ U.T - X).max() < 1e-12 * np.abs(X).max()
    f0b, Ub, svb, _, _ = emri.build_basis(F, 0)
    assert np.allclose(f0b, f0) and Ub.shape == (10, 0)


def _problem(n_seg=4, n_bins=33, pitch=40, dtype=0, n=10, top_k=2, k_min=0, k_max=-1, reserved=0):
    pb = emri._Problem()
    pb.power = _power(n_seg, n_bins, pitch, dtype)
    pb.f0 = pb.U = pb.coeffs = FAKE
    pb.n_tmpl = n
    pb.top_k = top_k
    pb.k_min, pb.k_max, pb.reserved = k_min, k_max, reserved
    pb.stat = pb.topk_val = pb.topk_idx = FAKE
    return pb


def test_batched_workspace_size_and_validation():
    lib = emri.load()
    arr = (emri._Problem * 3)(_problem(), _problem(n_seg=7, n=0, top_k=0), _problem(n_bins=100, pitch=104))
    nb = ctypes.c_size_t()
    assert lib.score_batched_workspace_size(arr, 3, 2, ctypes.byref(nb)) == 0 and nb.value > 0
    plan = emri._Plan()
    bad_cases = [
        ((emri._Problem * 1)(_problem(dtype=1)), 1, 2),          # fine alone ...
    ]
    mixed = (emri._Problem * 2)(_problem(), _problem(dtype=1))
    assert lib.score_batched_workspace_size(mixed, 2, 2, ctypes.byref(nb)) == -1     # mixed dtypes
    for bad in (_problem(top_k=5000), _problem(n=-1), _problem(k_min=3, k_max=2), _problem(reserved=1),
                _problem(pitch=36)):
        one = (emri._Problem * 1)(bad)
        assert lib.score_batched_workspace_size(one, 1, 2, ctypes.byref(nb)) == -1
        assert lib.score_batched_plan(one, 1, 2, None, FAKE, 1 << 30, ctypes.byref(plan), None) == -1
    assert lib.score_batched_workspace_size(arr, 3, 33, ctypes.byref(nb)) == -1
    opts = emri._BatchOpts(3, 0)
    assert lib.score_batched_plan(arr, 3, 2, ctypes.byref(opts), FAKE, 1 << 30, ctypes.byref(plan), None) == -1
    assert lib.score_batched_plan(arr, 3, 2, None, FAKE + 16, 1 << 30, ctypes.byref(plan), None) == -1
    assert lib.score_batched_run(ctypes.byref(emri._Plan()), None) == -1               # not a plan


def test_batched_tile_options():
    assert emri.batched_tile_options(8)[0] == 9 and len(emri.batched_tile_options(8)) == 2
    assert len(emri.batched_tile_options(5)) == 1


def test_mixed_precision_validation():
    lib = emri.load()
    nb = ctypes.c_size_t()
    pw = _power()
    assert lib.score_tracks_workspace_size(ctypes.byref(pw), 8, 10, 2, 0, ctypes.byref(nb)) == 0
    ws = 0x100000

    def call(K=8, precision=1, pitch=40, bins=None, reserved=0):
        p = _power(pitch=pitch)
        o = emri._Opts(0, -1, precision)
        o.reserved[0] = reserved
        return lib.score_tracks(ctypes.byref(p), FAKE, FAKE, K, FAKE, 10, 2, FAKE, FAKE, FAKE, bins, None,
                                ctypes.byref(o), ws, 1 << 30, None)
    assert call(K=0) == -5 and call(K=17) == -5          # built for 1 <= K <= 16
    assert call(precision=2) == -1                       # unknown precision
    assert call(bins=FAKE) == -5                         # no validation kernel for the mixed form
    assert call(reserved=1) == -1
    assert call(pitch=33) == -1                          # pitch not a multiple of 8
    opts = emri._BatchOpts(0, 0, 1)
    plan = emri._Plan()
    arr = (emri._Problem * 1)(_problem())
    assert lib.score_batched_plan(arr, 1, 17, ctypes.byref(opts), FAKE, 1 << 30, ctypes.byref(plan), None) == -5
    assert lib.score_batched_plan(arr, 1, 8, ctypes.byref(emri._BatchOpts(2, 0, 1)), FAKE, 1 << 30,
                                  ctypes.byref(plan), None) == -5      # four rows per step only
    assert lib.score_batched_plan(arr, 1, 8, ctypes.byref(emri._BatchOpts(0, 0, 3)), FAKE, 1 << 30,
                                  ctypes.byref(plan), None) == -1


def test_noalloc_limit_and_rejections():
    """score_tracks_noalloc validates like score_tracks and refuses, before any
    HIP call, a request whose workspace would not fit its static scratch."""
    lib = emri.load()
    limit = lib.score_tracks_noalloc_limit()
    assert limit == 4 << 20
    pw = _power(n_seg=192, n_bins=8193, pitch=8200)
    call = lambda n, stat, K=8, top_k=256: lib.score_tracks_noalloc(
        ctypes.byref(pw), FAKE, FAKE, K, FAKE, n, top_k, stat, FAKE, FAKE, None, None, None, None)
    need = ctypes.c_size_t(0)
    assert lib.score_tracks_workspace_size(ctypes.byref(pw), 8, 2_000_000, 256, 1, ctypes.byref(need)) == 0
    assert need.value > limit
    assert call(2_000_000, None) == -3                        # statistic in the scratch: too big
    assert b"static scratch" in lib.emri_last_error()
    assert call(33, FAKE, K=33) == -1
    assert call(-1, FAKE) == -1
    assert call(10, FAKE + 4) == -1


def _chain(n_walkers=16, n_seg=4, f0=FAKE, box=FAKE, coeffs=FAKE, reserved=0):
    from paper_2510_20891_amd import _Chain
    c = _Chain()
    c.power = _power(n_seg=n_seg)
    c.f0, c.U, c.box_lo, c.box_hi, c.coeffs, c.stat = f0, FAKE, box, box, coeffs, FAKE
    c.n_walkers, c.k_min, c.k_max, c.reserved = n_walkers, 0, -1, reserved
    return c


@pytest.mark.parametrize("kw,K,status", [
    (dict(n_walkers=2), 8, -1), (dict(), 0, -1), (dict(), 33, -1), (dict(f0=None), 8, -1),
    (dict(box=None), 8, -1), (dict(coeffs=FAKE + 4), 8, -1), (dict(reserved=1), 8, -1), (dict(n_seg=0), 8, -1),
])
def test_search_rejects(kw, K, status):
    """The search calls validate their chains before any HIP call."""
    lib = emri.load()
    arr = (emri._Chain * 1)(_chain(**kw))
    nb = ctypes.c_size_t(0)
    assert lib.search_workspace_size(arr, 1, K, ctypes.byref(nb)) == status
    assert lib.search_seed_workspace_size(arr, 1, K, 64, ctypes.byref(nb)) == status
    assert lib.emri_last_error()


def test_search_sizes_and_plan_arguments():
    lib = emri.load()
    arr = (emri._Chain * 2)(_chain(), _chain(n_walkers=40, n_seg=9))
    nb = ctypes.c_size_t(0)
    assert lib.search_workspace_size(arr, 2, 8, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.search_seed_workspace_size(arr, 2, 8, 64, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.search_seed_workspace_size(arr, 2, 8, 20, ctypes.byref(nb)) == -1     # 40 walkers of 20 draws
    plan = emri._SearchPlan()
    assert lib.search_generation(ctypes.byref(plan), FAKE, FAKE, FAKE, None, None) == -1   # not a plan
    assert lib.search_generations(ctypes.byref(plan), 2, FAKE, FAKE, FAKE, None) == -1     # not a plan
    assert lib.search_generations(None, 2, FAKE, FAKE, FAKE, None) == -1
    assert lib.search_plan(arr, 2, 8, None, FAKE + 16, 1 << 20, ctypes.byref(plan), None) == -1   # alignment
    assert lib.search_plan(arr, 2, 8, None, FAKE, 64, ctypes.byref(plan), None) == -3          # too small


@pytest.mark.parametrize("n_harm,ratios,K,status", [
    (0, [1.0], 8, -1), (5, [1.0] * 5, 8, -5), (2, [1.0, float("nan")], 8, -1), (2, [1.0, -0.5], 8, -1),
    (2, [1.0, 2000.0], 8, -1), (2, [1.0, 0.5], 17, -5), (2, [1.0, 0.5], 0, -5),
])
def test_harmonics_rejects(n_harm, ratios, K, status):
    lib = emri.load()
    pw = _power()
    rr = (ctypes.c_double * max(1, len(ratios)))(*ratios)
    st = lib.score_tracks_harmonics(ctypes.byref(pw), FAKE, FAKE, K, FAKE, 10, n_harm, rr, 4, FAKE, FAKE, FAKE,
                                    None, FAKE, 1 << 20, None)
    assert st == status
    assert lib.emri_last_error()


def test_harmonics_rejects_mixed_precision():
    lib = emri.load()
    pw = _power()
    rr = (ctypes.c_double * 2)(1.0, 0.5)
    opts = _Opts(0, -1, 1)
    assert lib.score_tracks_harmonics(ctypes.byref(pw), FAKE, FAKE, 8, FAKE, 10, 2, rr, 4, FAKE, FAKE, FAKE,
                                      ctypes.byref(opts), FAKE, 1 << 20, None) == -5
