"""Seeded synthetic inputs for the single-harmonic EMRI track search.

This module only draws inputs: noise time series, an injected chirping harmonic,
training frequency tracks and coefficient batches.  It holds none of the search
method's arithmetic (no SFT power, no basis, no scoring); the oracle and the GPU
library both consume what it returns.

The paper runs on LISA TDI-A data with EMRI signals from a trajectory model
(Sec. II F).  Those data and models are not available here, so every workload
is replaced by seeded stand-ins with the same structure:

* stationary Gaussian noise with a known one-sided PSD S(f) (white, or the
  coloured law S(f) = 1 + (f/3 mHz)^-4 + (f/20 mHz)^2);
* one chirping harmonic f(t) = f0 (1 - t/tau)^(-3/8) at a chosen SNR, standing in
  for the dominant m=2 harmonic of Eq. (2);
* training tracks drawn from the same chirp law sampled at the SFT midpoints,
  standing in for the 10^4 trajectory tracks of Sec. II C;
* coefficient vectors drawn uniformly inside the basis-projection box
  (Sec. II C, last paragraph; Sec. II D, initial population).

* the random numbers a population search draws (Sec. II D): seed candidates
  uniform in the box with initial frequencies uniform in a range, and for
  every differential-evolution generation the two partner walkers and the
  weight of each walker.

Seeds: ``rng(cfg, stream, purpose)`` with purpose 0 = noise, 1 = injection
parameters and phase, 2 = training tracks, 3 + 16*chunk = coefficient chunk
``chunk``, 4 = request arrivals and sizes, 5 = search seeding draws,
6 + 16*gen = the draws of search generation ``gen``.
"""
from __future__ import annotations

import math

import numpy as np

YEAR_S = 365.25 * 86400.0          # Julian year in seconds
COEFF_CHUNK = 1 << 16              # templates per seeded coefficient chunk

PURPOSE_NOISE = 0
PURPOSE_INJECTION = 1
PURPOSE_TRAINING = 2
PURPOSE_COEFF = 3
PURPOSE_REQUESTS = 4
PURPOSE_SEARCH_SEED = 5
PURPOSE_SEARCH_GEN = 6


def rng(cfg: int, stream: int, purpose: int) -> np.random.Generator:
    """Independent generator for (config, stream, purpose)."""
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(stream), int(purpose)]))


# --------------------------------------------------------------------------- PSDs
def psd_white(sigma: float, dt: float):
    """One-sided PSD of white noise of variance sigma^2 sampled every dt: 2 sigma^2 dt."""
    level = 2.0 * sigma * sigma * dt
    return lambda f: np.full_like(np.asarray(f, dtype=np.float64), level)


def psd_coloured(f):
    """S(f) = 1 + (f/3 mHz)^-4 + (f/20 mHz)^2 (infinite at f = 0)."""
    f = np.asarray(f, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return 1.0 + (f / 3e-3) ** -4 + (f / 20e-3) ** 2


def psd_on_bins(psd_fn, n_sft: int, dt: float) -> np.ndarray:
    """The PSD sampled at the SFT bin frequencies f_b = b / (n_sft dt), b = 0..n_sft/2."""
    t_sft = n_sft * dt
    return np.asarray(psd_fn(np.arange(n_sft // 2 + 1) / t_sft), dtype=np.float64)


# --------------------------------------------------------------------------- noise
def white_noise(n: int, sigma: float, g: np.random.Generator) -> np.ndarray:
    return sigma * g.standard_normal(n)


def coloured_noise(n: int, dt: float, psd_fn, g: np.random.Generator,
                   f_clamp: float = 1e-4) -> np.ndarray:
    """Gaussian noise with one-sided PSD psd_fn, by spectral shaping of white noise.

    Unit-variance white noise has one-sided PSD 2 dt, so its spectrum is scaled by
    sqrt(S(f) / (2 dt)).  DC is zeroed and S is held at S(f_clamp) below f_clamp,
    which keeps the f^-4 wall from putting a huge slow wander into every segment.
    """
    w = g.standard_normal(n)
    spec = np.fft.rfft(w)
    f = np.fft.rfftfreq(n, dt)
    s = np.asarray(psd_fn(np.maximum(f, f_clamp)), dtype=np.float64)
    spec *= np.sqrt(s / (2.0 * dt))
    spec[0] = 0.0
    return np.fft.irfft(spec, n)


# --------------------------------------------------------------------------- chirp
def chirp_frequency(t, f0: float, tau: float):
    """f(t) = f0 (1 - t/tau)^(-3/8): leading-order inspiral chirp law."""
    t = np.asarray(t, dtype=np.float64)
    return f0 * (1.0 - t / tau) ** (-0.375)


def chirp_phase(t, f0: float, tau: float):
    """Phi(t) = 2 pi f0 (8 tau / 5) [1 - (1 - t/tau)^(5/8)], the integral of 2 pi f(t)."""
    t = np.asarray(t, dtype=np.float64)
    return 2.0 * math.pi * f0 * (1.6 * tau) * (1.0 - (1.0 - t / tau) ** 0.625)


def optimal_snr(h: np.ndarray, dt: float, psd_fn) -> float:
    """rho^2 = 4 sum_b |h~_b|^2 df / S(f_b), h~ = dt FFT(h), df = 1/T_obs.

    The inner-product normalisation is the one the paper uses for <.|.> (Eq. (7));
    the paper does not spell out its SNR, so the matched-filter convention is taken.
    """
    n = h.size
    hf = dt * np.fft.rfft(h)
    f = np.fft.rfftfreq(n, dt)
    s = np.asarray(psd_fn(f), dtype=np.float64)
    ok = np.isfinite(s) & (s > 0)
    df = 1.0 / (n * dt)
    return math.sqrt(4.0 * df * float(np.sum(np.abs(hf[ok]) ** 2 / s[ok])))


def injection(n: int, dt: float, f0: float, tau: float, snr: float, psd_fn,
              phi0: float, t_cut: float | None = None) -> np.ndarray:
    """A cos(Phi(t) + phi0), t = k dt, scaled to the requested SNR.

    The signal is cut (set to zero) from plunge (t >= tau, or t >= t_cut when
    given) and wherever its frequency exceeds 0.45/dt, so nothing aliases.
    """
    t = np.arange(n) * dt
    live = t < (tau if t_cut is None else min(tau, t_cut))
    h = np.zeros(n)
    tl = t[live]
    f = chirp_frequency(tl, f0, tau)
    keep = f <= 0.45 / dt
    h_live = np.where(keep, np.cos(chirp_phase(tl, f0, tau) + phi0), 0.0)
    h[live] = h_live
    rho = optimal_snr(h, dt, psd_fn)
    if snr <= 0 or rho == 0.0:
        return np.zeros(n)
    return h * (snr / rho)


# --------------------------------------------------------------------------- tracks
def segment_midpoints(n_seg: int, t_sft: float) -> np.ndarray:
    """t_alpha = (alpha + 1/2) T_SFT, time origin at the first sample."""
    return (np.arange(n_seg) + 0.5) * t_sft


def training_tracks(n_train: int, t_mid: np.ndarray, f0_range, tau_range,
                    g: np.random.Generator) -> np.ndarray:
    """[n_train, n_seg] chirp tracks with f0 ~ U[f0_range], tau ~ U[tau_range] (seconds)."""
    f0 = g.uniform(f0_range[0], f0_range[1], n_train)
    tau = g.uniform(tau_range[0], tau_range[1], n_train)
    return f0[:, None] * (1.0 - t_mid[None, :] / tau[:, None]) ** (-0.375)


def plunge_tracks(n_train: int, t_mid: np.ndarray, t_plunge: float, fp_range, tc_range,
                  g: np.random.Generator) -> np.ndarray:
    """[n_train, n_seg] tracks that plunge at t_plunge: the chirp law with
    coalescence time t_plunge + t_c, cut at the plunge,
    f(t) = f_p (1 + (t_plunge - t) / t_c)^(-3/8)  (t <= t_plunge),
    with f_p ~ U[fp_range] (Hz, the frequency at plunge) and t_c ~ logU[tc_range]
    (seconds).  Stand-ins for trajectory tracks that all end at one plunge time."""
    fp = g.uniform(fp_range[0], fp_range[1], n_train)
    tc = np.exp(g.uniform(math.log(tc_range[0]), math.log(tc_range[1]), n_train))
    return fp[:, None] * (1.0 + (t_plunge - t_mid[None, :]) / tc[:, None]) ** (-0.375)


def coefficient_chunk(cfg: int, stream: int, chunk: int, n: int,
                      box_lo: np.ndarray, box_hi: np.ndarray) -> np.ndarray:
    """``n`` FP32 coefficient vectors uniform in the box, from seeded chunk ``chunk``.

    Drawn in FP64 and rounded once to FP32; the FP32 values are the canonical
    input that every implementation widens exactly.
    """
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    g = rng(cfg, stream, PURPOSE_COEFF + 16 * int(chunk))
    return g.uniform(lo, hi, size=(int(n), lo.size)).astype(np.float32)


def coefficients(cfg: int, stream: int, n: int, box_lo, box_hi,
                 chunk: int = COEFF_CHUNK) -> np.ndarray:
    """``n`` coefficient vectors assembled from consecutive seeded chunks."""
    k = len(box_lo)
    out = np.empty((int(n), k), dtype=np.float32)
    for c, start in enumerate(range(0, int(n), chunk)):
        m = min(chunk, int(n) - start)
        out[start:start + m] = coefficient_chunk(cfg, stream, c, m, box_lo, box_hi)
    return out


def coefficients_rows(cfg: int, stream: int, rows: np.ndarray, box_lo, box_hi,
                      chunk: int = COEFF_CHUNK) -> np.ndarray:
    """The coefficient vectors at template indices ``rows`` (regenerated chunk by chunk)."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty((rows.size, len(box_lo)), dtype=np.float32)
    for c in np.unique(rows // chunk):
        sel = np.nonzero(rows // chunk == c)[0]
        full = coefficient_chunk(cfg, stream, int(c), chunk, box_lo, box_hi)
        out[sel] = full[rows[sel] - c * chunk]
    return out


# --------------------------------------------------------------------------- configs
def stream_config0(stream: int = 0) -> dict:
    """Tiny plain-method stream: 30 days of unit white noise at 10 s, 1-day SFTs."""
    cfg, dt, n, n_sft = 0, 10.0, 259_200, 8640
    gi = rng(cfg, stream, PURPOSE_INJECTION)
    phi0 = gi.uniform(0.0, 2.0 * math.pi)
    psd_fn = psd_white(1.0, dt)
    x = white_noise(n, 1.0, rng(cfg, stream, PURPOSE_NOISE))
    inj = dict(f0=5e-3, tau=2.0 * YEAR_S, snr=30.0, phi0=phi0)
    x = x + injection(n, dt, inj["f0"], inj["tau"], inj["snr"], psd_fn, phi0)
    n_seg = n // n_sft
    t_mid = segment_midpoints(n_seg, n_sft * dt)
    tracks = training_tracks(1000, t_mid, (2e-3, 10e-3), (0.5 * YEAR_S, 5.0 * YEAR_S),
                             rng(cfg, stream, PURPOSE_TRAINING))
    return dict(cfg=cfg, stream=stream, dt=dt, n_sft=n_sft, x=x, psd_fn=psd_fn,
                psd=psd_on_bins(psd_fn, n_sft, dt), tracks=tracks, K=4, n_tmpl=4096,
                top_k=16, injection=inj, t_mid=t_mid)


def stream_config1(stream: int = 0, cfg: int = 1, duration_s: float = 3.15e7,
                   snr: float | None = 30.0) -> dict:
    """One year (3.15e7 s) of coloured noise at 10 s, SFTs of 16384 samples."""
    dt, n_sft = 10.0, 16384
    n = int(round(duration_s / dt))
    gi = rng(cfg, stream, PURPOSE_INJECTION)
    f0 = gi.uniform(1e-3, 20e-3)
    tau = gi.uniform(1.0, 10.0) * YEAR_S
    phi0 = gi.uniform(0.0, 2.0 * math.pi)
    x = coloured_noise(n, dt, psd_coloured, rng(cfg, stream, PURPOSE_NOISE))
    inj = None
    if snr is not None and snr > 0:
        inj = dict(f0=f0, tau=tau, snr=float(snr), phi0=phi0)
        x = x + injection(n, dt, f0, tau, snr, psd_coloured, phi0)
    n_seg = n // n_sft
    t_mid = segment_midpoints(n_seg, n_sft * dt)
    tracks = training_tracks(5000, t_mid, (1e-3, 20e-3), (1.0 * YEAR_S, 10.0 * YEAR_S),
                             rng(cfg, stream, PURPOSE_TRAINING))
    return dict(cfg=cfg, stream=stream, dt=dt, n_sft=n_sft, x=x, psd_fn=psd_coloured,
                psd=psd_on_bins(psd_coloured, n_sft, dt), tracks=tracks, K=8,
                n_tmpl=10_000_000, top_k=256, injection=inj, t_mid=t_mid)


def stream_progressive(stream: int = 0, cfg: int = 6, plunge_frac: float = 0.7, snr: float | None = 30.0) -> dict:
    """The progressive-duration search's stand-in: one year of config-1 noise
    (3.15e7 s at 10 s, SFTs of 16384 samples, 192 segments) holding one
    harmonic that plunges inside the year, at plunge_frac of the data, with
    f_p ~ U[8, 30] mHz and t_c ~ logU[0.02, 1] yr; training tracks (5000, the
    same law) plunge at the end of the data, so a basis shifted by whole
    segments aligns the plunge with the end of any shorter duration."""
    dt, n_sft = 10.0, 16384
    n = int(round(3.15e7 / dt))
    n_seg = n // n_sft
    t_sft = n_sft * dt
    gi = rng(cfg, stream, PURPOSE_INJECTION)
    fp = gi.uniform(8e-3, 30e-3)
    tc = math.exp(gi.uniform(math.log(0.02 * YEAR_S), math.log(1.0 * YEAR_S)))
    phi0 = gi.uniform(0.0, 2.0 * math.pi)
    t_inj = plunge_frac * n_seg * t_sft
    tau = t_inj + tc
    f0 = fp * (1.0 + t_inj / tc) ** (-0.375)                  # frequency at t = 0
    x = coloured_noise(n, dt, psd_coloured, rng(cfg, stream, PURPOSE_NOISE))
    inj = None
    if snr is not None and snr > 0:
        inj = dict(f0=f0, tau=tau, t_plunge=t_inj, f_plunge=fp, t_c=tc, snr=float(snr), phi0=phi0)
        x = x + injection(n, dt, f0, tau, snr, psd_coloured, phi0, t_cut=t_inj)
    t_mid = segment_midpoints(n_seg, t_sft)
    tracks = plunge_tracks(5000, t_mid, n_seg * t_sft, (8e-3, 30e-3), (0.02 * YEAR_S, 1.0 * YEAR_S),
                           rng(cfg, stream, PURPOSE_TRAINING))
    return dict(cfg=cfg, stream=stream, dt=dt, n_sft=n_sft, x=x, psd_fn=psd_coloured,
                psd=psd_on_bins(psd_coloured, n_sft, dt), tracks=tracks, K=8, injection=inj, t_mid=t_mid)


def batched_streams(n_streams: int = 64, cfg: int = 3) -> list[dict]:
    """Uneven streams: duration U[3, 12] months, an injection with probability 1/2 at SNR U[20, 40],
    template count floor(logU[1e5, 1e7])."""
    out = []
    for s in range(n_streams):
        g = rng(cfg, s, PURPOSE_REQUESTS)
        months = g.uniform(3.0, 12.0)
        has_inj = g.uniform() < 0.5
        snr = g.uniform(20.0, 40.0)
        n_tmpl = int(math.floor(math.exp(g.uniform(math.log(1e5), math.log(1e7)))))
        st = stream_config1(stream=s, cfg=cfg, duration_s=months * YEAR_S / 12.0,
                            snr=snr if has_inj else None)
        st["n_tmpl"] = n_tmpl
        out.append(st)
    return out


def serving_requests(n_streams: int = 16, rate: float = 2000.0, seconds: float = 32.0, cfg: int = 4,
                     pool_size: int = 1 << 22, top_k: int = 32) -> list[dict]:
    """Poisson arrivals at ``rate`` per second for ``seconds``; each request draws a
    template count floor(logU[256, 65536]), a stream uniform over ``n_streams``, and
    an offset into a shared pool of ``pool_size`` coefficient vectors (the pool is
    ``coefficients(cfg, 0, pool_size, ...)``; rows are reused across requests)."""
    g = rng(cfg, 0, PURPOSE_REQUESTS)
    out, t, rid = [], 0.0, 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= seconds:
            break
        n = int(math.floor(math.exp(g.uniform(math.log(256.0), math.log(65536.0)))))
        out.append(dict(rid=rid, t=t, stream=int(g.integers(0, n_streams)), n=n,
                        offset=int(g.integers(0, pool_size - n + 1)), top_k=top_k))
        rid += 1
    return out


def device_coefficients(cfg: int, stream: int, n: int, box_lo, box_hi, device="cuda"):
    """``n`` coefficient vectors uniform in the box, drawn on the GPU (torch's
    Philox generator seeded with (cfg, stream)); for benchmark batches too large
    to draw on the host.  Same law as ``coefficients``, different stream of numbers."""
    import torch
    lo = torch.as_tensor(np.asarray(box_lo, dtype=np.float64), device=device)
    hi = torch.as_tensor(np.asarray(box_hi, dtype=np.float64), device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(1_000_003 * int(cfg) + int(stream))
    out = torch.empty((int(n), lo.numel()), dtype=torch.float32, device=device)
    step = 1 << 22
    for s in range(0, int(n), step):
        m = min(step, int(n) - s)
        u = torch.rand((m, lo.numel()), dtype=torch.float64, device=device, generator=gen)
        out[s:s + m] = (lo + u * (hi - lo)).to(torch.float32)
    return out


# ----------------------------------------------------------------- search draws
def search_seed_draws(cfg: int, chain: int, n: int, box_lo, box_hi, f_lo: float = 5e-4, f_hi: float = 1e-2):
    """Seed candidates of one search chain: coefficient vectors uniform in the
    box (drawn in FP64, stored FP32) and initial frequencies uniform in
    [f_lo, f_hi] Hz (FP64)."""
    g = rng(cfg, chain, PURPOSE_SEARCH_SEED)
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    c = (lo[None, :] + (hi - lo)[None, :] * g.random((n, lo.size))).astype(np.float32)
    return c, g.uniform(f_lo, f_hi, n)


def search_generation_draws(cfg: int, chain: int, gen: int, n: int, f_lo: float = 0.3, f_hi: float = 1.5):
    """Partners and weights of one differential-evolution generation: for every
    walker i two other walkers r1 != r2 (uniform over the walkers other than i,
    then over those other than i and r1) and a weight F uniform in [f_lo, f_hi]."""
    if n < 3:
        raise ValueError("a generation needs at least three walkers")
    g = rng(cfg, chain, PURPOSE_SEARCH_GEN + 16 * gen)
    i = np.arange(n)
    r1 = (i + 1 + g.integers(0, n - 1, n)) % n
    u = g.integers(0, n - 2, n)
    a, b = np.minimum(i, r1), np.maximum(i, r1)
    r2 = u + (u >= a)
    r2 = r2 + (r2 >= b)
    F = g.uniform(f_lo, f_hi, n)
    return r1.astype(np.int32), r2.astype(np.int32), F


def device_generation_draws(cfg: int, n_gen: int, walkers: list, device="cuda", f_lo: float = 0.3, f_hi: float = 1.5):
    """Partners and weights of n_gen generations for chains of the given walker
    counts (concatenated), drawn on the GPU (torch's Philox generator seeded
    with cfg); the same law as ``search_generation_draws``, for benchmark runs.
    Returns int32 r1, r2 and float64 F tensors of shape (n_gen, sum(walkers))."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(2_000_003 * int(cfg) + 17)
    n = torch.cat([torch.full((w,), int(w), dtype=torch.int64, device=device) for w in walkers])
    i = torch.cat([torch.arange(w, dtype=torch.int64, device=device) for w in walkers])
    tot = int(n.numel())
    u1 = torch.rand((n_gen, tot), dtype=torch.float64, device=device, generator=gen)
    u2 = torch.rand((n_gen, tot), dtype=torch.float64, device=device, generator=gen)
    r1 = (i + 1 + torch.floor(u1 * (n - 1)).to(torch.int64)) % n
    u = torch.floor(u2 * (n - 2)).to(torch.int64)
    a, b = torch.minimum(i, r1), torch.maximum(i, r1)
    r2 = u + (u >= a).to(torch.int64)
    r2 = r2 + (r2 >= b).to(torch.int64)
    F = f_lo + (f_hi - f_lo) * torch.rand((n_gen, tot), dtype=torch.float64, device=device, generator=gen)
    return r1.to(torch.int32), r2.to(torch.int32), F
