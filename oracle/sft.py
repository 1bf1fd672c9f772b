"""Oracle: PSD-normalised SFT power (test infrastructure only).

The data stream is cut into consecutive, non-overlapping segments of n_sft
samples (T_SFT = n_sft dt, frequency resolution 1/T_SFT; Sec. II B).  Each
segment is windowed and Fourier transformed; the power in bin b is divided by
the known PSD at f_b = b / T_SFT (Eq. (7) weights every bin by 1/S_n(f_k), and
the PSD is taken as known, Sec. II F).

Readings where the paper is silent:
* window: periodic Hann w_n = sin^2(pi n / N), no overlap, no detrending;
* normalisation: |X_b|^2 / (sum_n w_n^2 * S(f_b) / (2 dt)), which makes the
  noise-only power exactly Exp(1) in bins 2..N/2-2 (so the nearest-bin
  statistic over N_seg segments is Gamma(N_seg, 1));
* a bin whose PSD is non-positive or non-finite gets power 0;
* the samples after the last whole segment are dropped.
"""
from __future__ import annotations

import numpy as np


def hann_periodic(n: int) -> np.ndarray:
    """w_k = sin^2(pi k / n), k = 0..n-1 (the DFT-even Hann window)."""
    return np.sin(np.pi * np.arange(n) / n) ** 2


def sft_bin_frequencies(n_sft: int, dt: float) -> np.ndarray:
    return np.arange(n_sft // 2 + 1) / (n_sft * dt)


def segments(x: np.ndarray, n_sft: int) -> np.ndarray:
    """Consecutive non-overlapping segments, shape (n_seg, n_sft); the tail is dropped."""
    n_seg = x.size // n_sft
    return x[: n_seg * n_sft].reshape(n_seg, n_sft)


def normaliser(w: np.ndarray, psd: np.ndarray, dt: float) -> np.ndarray:
    """sum_n w_n^2 * S(f_b) / (2 dt): the noise-only expectation of |X_b|^2."""
    return np.sum(w * w) * psd / (2.0 * dt)


def build_sfts(x, dt: float, n_sft: int, psd) -> np.ndarray:
    """Normalised power P[alpha, b], shape (n_seg, n_sft/2 + 1), FP64.

    x   : real time series, FP64, sample spacing dt seconds
    psd : one-sided PSD at f_b = b/(n_sft dt), b = 0..n_sft/2
    """
    x = np.asarray(x, dtype=np.float64)
    psd = np.asarray(psd, dtype=np.float64)
    n_sft = int(n_sft)
    if n_sft < 4 or n_sft % 2:
        raise ValueError("n_sft must be even and >= 4")
    n_bins = n_sft // 2 + 1
    if psd.shape != (n_bins,):
        raise ValueError("psd must have n_sft/2 + 1 entries")
    w = hann_periodic(n_sft)
    spec = np.fft.rfft(segments(x, n_sft) * w[None, :], axis=1)
    power = spec.real ** 2 + spec.imag ** 2
    ok = np.isfinite(psd) & (psd > 0)
    denom = normaliser(w, np.where(ok, psd, 1.0), dt)
    return np.where(ok[None, :], power / denom[None, :], 0.0)
