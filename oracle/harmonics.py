"""Oracle: the multi-harmonic statistic (test infrastructure only).

Sec. IV proposes including several harmonics of the EMRI signal, with a cost
that grows in proportion to their number.  Reading (the paper gives no
formula): harmonic h follows the track scaled by a fixed frequency ratio r_h
(r = 1 is the searched, dominant harmonic; for the m-harmonics of a circular
orbit with m = 2 dominant, r = m / 2), each harmonic's per-segment statistic
is the nearest-bin normalised power of its own track, and the statistic sums
them over harmonics and segments:

    x[j, alpha]     = (f0[alpha] + sum_k c[j, k] U[alpha, k]) T_SFT   (FP64)
    b_h[j, alpha]   = rint(r_h x[j, alpha])                          (half to even)
    S[j]            = sum_h sum_alpha P[alpha, b_h] [k_min <= b_h <= k_max]

The scaled position r_h x is formed in FP64 before rounding.  With one
harmonic of ratio 1 this is the single-harmonic statistic.
"""
from __future__ import annotations

import numpy as np

from .score import chosen_bins, near_tie_mask, topk_order, track_positions


def harmonic_positions(x, ratios) -> np.ndarray:
    """r_h x for every harmonic: shape (H, n_tmpl, n_seg), FP64."""
    r = np.asarray(ratios, dtype=np.float64)
    return r[:, None, None] * np.asarray(x, dtype=np.float64)[None, :, :]


def score_harmonics(P, f0, U, coeffs, t_sft: float, ratios, top_k: int = 0, k_min: int = 0, k_max=None,
                    chunk: int = 32768):
    """Multi-harmonic statistic, top-k by (-S, index) and, per template, whether
    any harmonic position lies within the near-tie band of a half-integer."""
    P = np.asarray(P, dtype=np.float64)
    n_seg, n_bins = P.shape
    coeffs = np.asarray(coeffs, dtype=np.float32)
    Um = np.asarray(U, dtype=np.float64).reshape(n_seg, -1)
    n = coeffs.shape[0]
    stat = np.zeros(n)
    near = np.zeros(n, dtype=bool)
    rows = np.arange(n_seg)[None, :]
    for s in range(0, n, chunk):
        x = track_positions(f0, Um, coeffs[s:s + chunk], t_sft)
        xh = harmonic_positions(x, ratios)
        for h in range(xh.shape[0]):
            b, valid = chosen_bins(xh[h], n_bins, k_min, k_max)
            stat[s:s + chunk] += np.where(valid, P[rows, np.where(valid, b, 0)], 0.0).sum(axis=1)
            near[s:s + chunk] |= near_tie_mask(xh[h]).any(axis=1)
    vals, idx = topk_order(stat, top_k)
    return dict(stat=stat, topk_val=vals, topk_idx=idx, near=near)
