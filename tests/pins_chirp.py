"""Checks that pin the linear-chirp statistic oracle (Sec. II B, Eqs. (4)-(7)).

Each check takes the function under test, so the same checks run against the
oracle (they must pass) and against planted mistakes (one must fail).

* Template SFT against a brute-force DFT: the N-point DFT of a sampled,
  periodic-Hann-windowed linear chirp exp(i[2 pi f (t - t_a) + pi fdot (t - t_a)^2])
  is N (-1)^k R(f T - k, fdot T^2) in the bins around f T, up to the
  discretisation of the integral.
* Without a frequency derivative the template is the Hann response in closed
  form, (1/2) sinc(d) + (1/4) sinc(d + 1) + (1/4) sinc(d - 1).
* One bin (P = 0): the statistic is the nearest-bin power |Z_k0|^2, whatever
  the template.
* A noiseless linear chirp A cos(phase) injected in a segment, scored with
  its own f and fdot, gives the matched-filter value in closed form,
  (4 A^2 N dt / 3) sum_k |R_k|^2 / S_k over the window (with a PSD that is
  not flat, so the 1/S weighting is pinned), and a template off by half a
  bin scores less.
* Finite differences of the track are exact for quadratic tracks; segments
  beyond the fddot validity limit, below the frequency cut-off or the
  derivative cut-off contribute nothing.
"""
from __future__ import annotations

import math

import numpy as np


def _sinc(x):
    return np.sinc(x)                    # sin(pi x) / (pi x)


def check_template_bruteforce(chirp_template_bins):
    N, P = 4096, 30
    n = np.arange(N)
    w = np.sin(np.pi * n / N) ** 2
    for k0, d0, beta in ((700, 0.31, 7.3), (1200, -0.45, -3.1), (900, 0.0, 0.0), (1500, 0.12, 22.0)):
        fT = k0 + d0
        u = n / N - 0.5                       # (t - t_a) / T, t_a the segment midpoint
        h = w * np.exp(1j * (2 * np.pi * fT * u + np.pi * beta * u * u))
        ks = k0 + np.arange(-P, P + 1)
        dft = np.array([np.sum(h * np.exp(-2j * np.pi * k * n / N)) for k in ks])
        R = chirp_template_bins(d0, beta, P)
        want = N * np.where(ks % 2 == 0, 1.0, -1.0) * R
        scale = np.abs(dft).max()
        assert np.abs(dft - want).max() <= 2e-6 * scale, (k0, d0, beta, np.abs(dft - want).max() / scale)


def check_template_no_derivative(chirp_template_bins):
    for d0 in (0.0, 0.2, -0.5, 0.37):
        P = 12
        m = np.arange(-P, P + 1)
        d = d0 - m
        want = 0.5 * _sinc(d) + 0.25 * _sinc(d + 1) + 0.25 * _sinc(d - 1)
        got = chirp_template_bins(d0, 0.0, P)
        assert np.abs(got - want).max() <= 1e-13, (d0, np.abs(got - want).max())


def check_one_bin_is_nearest_bin_power(score_chirp, build_sfts_complex, inverse_sqrt_psd):
    g = np.random.default_rng(71)
    n_sft, dt, n_seg, K = 512, 10.0, 6, 2
    x = g.standard_normal(n_sft * n_seg)
    psd = np.full(n_sft // 2 + 1, 20.0)
    Z = build_sfts_complex(x, dt, n_sft, psd)
    T = n_sft * dt
    f0 = np.linspace(40, 60, n_seg) / T
    U = g.standard_normal((n_seg, K)) * 2.0 / T
    C = g.uniform(-1, 1, (5, K)).astype(np.float32)
    res = score_chirp(Z, inverse_sqrt_psd(psd), f0, U, C, T, p_half=0, f_min=-np.inf, fdot_min=-np.inf)
    f = f0[None, :] + C.astype(np.float64) @ U.T
    k0 = np.rint(f * T).astype(int)
    want = np.abs(Z[np.arange(n_seg)[None, :], k0]) ** 2
    ok = res["valid"]
    assert np.allclose(res["per_segment"][ok], want[ok], rtol=1e-12, atol=0)
    assert ok.sum() > 0
    # a central bin outside the row: no contribution, even where window bins reach into the row
    Zr = Z[0]
    n_bins = Zr.shape[0]
    assert segment_statistic_of(score_chirp)(Zr, inverse_sqrt_psd(psd), (n_bins + 3) / T, 0.0, T, 10) == 0.0
    assert segment_statistic_of(score_chirp)(Zr, inverse_sqrt_psd(psd), -4.0 / T, 0.0, T, 10) == 0.0
    assert segment_statistic_of(score_chirp)(Zr, inverse_sqrt_psd(psd), (n_bins - 2) / T, 0.0, T, 10) > 0.0


def segment_statistic_of(score_chirp):
    import importlib
    return importlib.import_module(score_chirp.__module__).segment_statistic


def check_matched_chirp(segment_statistic, build_sfts_complex, inverse_sqrt_psd, chirp_template_bins):
    N, dt, P, A = 2048, 5.0, 40, 0.7
    T = N * dt
    n_bins = N // 2 + 1
    psd = 2.0 + 3.0 * (np.arange(n_bins) % 3)                 # not flat: the 1/S weighting matters
    for fT, beta in ((300.4, 6.5), (512.0, 0.0), (401.2, -4.0)):
        f, fdot = fT / T, beta / T ** 2
        t = np.arange(N) * dt
        phase = 2 * math.pi * f * (t - T / 2) + math.pi * fdot * (t - T / 2) ** 2 + 0.3
        x = A * np.cos(phase)
        Z = build_sfts_complex(x, dt, N, psd)[0]
        isq = inverse_sqrt_psd(psd)
        got = segment_statistic(Z, isq, f, fdot, T, P)
        k0 = int(np.rint(fT))
        R = chirp_template_bins(fT - k0, beta, P)
        k = k0 + np.arange(-P, P + 1)
        want = 4.0 * A * A * N * dt / 3.0 * np.sum(np.abs(R) ** 2 / psd[k])
        assert abs(got - want) <= 2e-4 * want, (fT, beta, got, want)
        off = segment_statistic(Z, isq, f + 0.5 / T, fdot, T, P)
        assert off < 0.9 * got


def check_track_derivatives(track_derivatives):
    T = 1000.0
    t = (np.arange(9) + 0.5) * T
    a, b, c = 1e-2, 3e-9, 2e-15
    f = (a + b * t + c * t * t)[None, :]
    fd, fdd = track_derivatives(f, T)
    assert np.allclose(fd[0], b + 2 * c * t, rtol=1e-10, atol=0)
    assert np.allclose(fdd[0], 2 * c, rtol=1e-6, atol=0)


def check_validity_and_cutoffs(score_chirp, build_sfts_complex, inverse_sqrt_psd):
    g = np.random.default_rng(72)
    n_sft, dt, n_seg = 1024, 10.0, 8
    T = n_sft * dt
    psd = np.full(n_sft // 2 + 1, 20.0)
    Z = build_sfts_complex(g.standard_normal(n_sft * n_seg), dt, n_sft, psd)
    isq = inverse_sqrt_psd(psd)
    tm = (np.arange(n_seg) + 0.5) * T
    # basis columns: a constant, a slope and a curvature (bins, per segment)
    U = np.stack([np.ones(n_seg), tm / T, (tm / T) ** 2], axis=1) / T
    f0 = np.full(n_seg, 60.0 / T)
    C = np.array([[0.0, 0.5, 0.0],      # fdot = 0.5 / T^2 > 0: valid everywhere
                  [0.0, -0.5, 0.0],     # fdot < 0: below the derivative cut-off everywhere
                  [0.0, 0.5, 3.5],      # fddot = 7 / T^3: |fddot| T^3 / 6 > 1, no segment
                  [0.0, 0.5, 2.5],      # fddot = 5 / T^3: still valid
                  [-57.0, 0.5, 0.0]],   # 3.25 .. 6.75 bins: below the 5-bin cut-off at first
                 dtype=np.float32)
    res = score_chirp(Z, isq, f0, U, C, T, p_half=10, f_min=5.0 / T, fdot_min=0.0)
    v = res["valid"]
    assert np.all(v[0]) and not np.any(v[1]) and not np.any(v[2]) and np.all(v[3])
    assert list(v[4]) == [False] * 4 + [True] * 4
    assert np.all(res["per_segment"][~v] == 0.0) and np.all(res["per_segment"][v] > 0.0)
    assert np.allclose(res["stat"], res["per_segment"].sum(axis=1))
