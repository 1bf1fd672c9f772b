"""Pins of the synthetic input generators and of the oracle on the tiny stream (CPU only)."""
import math

import numpy as np
from scipy import stats

import oracle
import synth


def test_chirp_phase_is_integral_of_frequency():
    f0, tau = 5e-3, 2 * synth.YEAR_S
    t = np.linspace(0, 0.9 * tau, 50)
    h = 1.0
    dphi = (synth.chirp_phase(t + h, f0, tau) - synth.chirp_phase(t - h, f0, tau)) / (2 * h)
    assert np.allclose(dphi, 2 * math.pi * synth.chirp_frequency(t, f0, tau), rtol=1e-7)
    assert synth.chirp_phase(0.0, f0, tau) == 0.0


def test_injection_snr():
    psd = synth.psd_white(1.0, 10.0)
    h = synth.injection(86400, 10.0, 5e-3, synth.YEAR_S, 30.0, psd, 0.3)
    assert abs(synth.optimal_snr(h, 10.0, psd) - 30.0) < 1e-9


def test_coloured_noise_matches_psd():
    dt, n_sft = 10.0, 16384
    x = synth.coloured_noise(40 * n_sft, dt, synth.psd_coloured, synth.rng(9, 0, 0))
    psd = synth.psd_on_bins(synth.psd_coloured, n_sft, dt)
    P = oracle.build_sfts(x, dt, n_sft, psd)
    f = oracle.sft_bin_frequencies(n_sft, dt)
    band = (f > 5e-4) & (f < 4.5e-2)
    mean = P[:, band].mean()
    assert abs(mean - 1.0) < 0.01
    # per octave as well
    for lo in (5e-4, 2e-3, 8e-3, 3e-2):
        sel = (f > lo) & (f < 1.5 * lo)
        assert abs(P[:, sel].mean() - 1.0) < 0.05


def test_coefficient_chunks_are_consistent():
    lo, hi = np.array([-1.0, 0.0]), np.array([1.0, 2.0])
    full = synth.coefficients(5, 0, 3 * 1000 + 17, lo, hi, chunk=1000)
    rows = np.array([0, 999, 1000, 2500, 3016])
    assert np.array_equal(synth.coefficients_rows(5, 0, rows, lo, hi, chunk=1000), full[rows])
    assert full.dtype == np.float32
    assert np.all(full >= lo.astype(np.float32)) and np.all(full <= hi.astype(np.float32))


def test_injection_recovered_tiny_stream():
    """Config-0 stream: the injected chirp's projected coefficients beat the noise law."""
    st = synth.stream_config0()
    P = oracle.build_sfts(st["x"], st["dt"], st["n_sft"], st["psd"])
    assert P.shape == (30, 4321)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], st["K"])
    inj = st["injection"]
    true_track = synth.chirp_frequency(st["t_mid"], inj["f0"], inj["tau"])
    c = (U.T @ (true_track - f0)).astype(np.float32)[None, :]
    t_sft = st["n_sft"] * st["dt"]
    # the basis reproduces the true track to well under a bin
    x_true = true_track * t_sft
    x_rec = oracle.track_positions(f0, U, c, t_sft)[0]
    assert np.abs(x_rec - x_true).max() < 1e-3
    C = synth.coefficients(0, 0, st["n_tmpl"], lo, hi)
    res = oracle.score_tracks(P, f0, U, np.vstack([C, c]), t_sft, st["top_k"])
    s_true = res["stat"][-1]
    assert s_true > stats.gamma(30).ppf(0.999)
    assert res["topk_idx"][0] == st["n_tmpl"]
    # random templates in the box look like noise on average
    assert abs(np.median(res["stat"][:-1]) - 30) < 5


def test_search_draws():
    lo, hi = np.array([-1.0, 0.0, 2.0]), np.array([1.0, 0.5, 3.0])
    c, f = synth.search_seed_draws(0, 2, 1000, lo, hi)
    assert c.dtype == np.float32 and c.shape == (1000, 3)
    assert np.all(c >= lo.astype(np.float32)) and np.all(c <= hi.astype(np.float32))
    assert np.all((f >= 5e-4) & (f <= 1e-2))
    for n in (3, 4, 17, 512):
        r1, r2, F = synth.search_generation_draws(0, 1, 3, n)
        i = np.arange(n)
        assert np.all((r1 != i) & (r2 != i) & (r1 != r2))
        assert r1.min() >= 0 and r2.min() >= 0 and r1.max() < n and r2.max() < n
        assert np.all((F >= 0.3) & (F <= 1.5))
    a = synth.search_generation_draws(0, 1, 3, 64)
    b = synth.search_generation_draws(0, 1, 4, 64)
    assert not np.array_equal(a[0], b[0])            # generations draw independently


def test_plunge_tracks_end_at_the_plunge():
    t_mid = synth.segment_midpoints(192, 163840.0)
    T = 192 * 163840.0
    F = synth.plunge_tracks(50, t_mid, T, (8e-3, 30e-3), (0.02 * synth.YEAR_S, synth.YEAR_S), synth.rng(0, 0, 2))
    assert F.shape == (50, 192)
    assert np.all(np.diff(F, axis=1) > 0)                       # chirping up to the plunge
    assert np.all(F[:, -1] <= 30e-3) and np.all(F[:, -1] >= 0.9 * 8e-3)
    assert np.all(F < 0.45 / 10.0)                              # below Nyquist at dt = 10 s


def test_progressive_stream_injection_stops_at_plunge():
    st = synth.stream_progressive(stream=0, plunge_frac=0.7)
    inj = st["injection"]
    assert abs(inj["t_plunge"] - 0.7 * 192 * 163840.0) < 1.0
    noise = synth.stream_progressive(stream=0, plunge_frac=0.7, snr=None)["x"]
    h = st["x"] - noise
    k = int(inj["t_plunge"] / st["dt"])
    assert np.all(h[k + 1:] == 0.0) and np.any(h[:k] != 0.0)
    assert np.isclose(synth.chirp_frequency(inj["t_plunge"] - 1e-6, inj["f0"], inj["tau"]), inj["f_plunge"],
                      rtol=1e-9)
