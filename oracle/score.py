"""Oracle: nearest-bin semi-coherent statistic and top-k (test infrastructure only).

Eq. (6) sums a per-segment statistic over segments; Eq. (7) maximises each
segment's inner product over phase.  For a template whose SFT is concentrated
in a single bin (the zero-bandwidth limit of the linear-chirp template of
Sec. II B), the per-segment term reduces to a fixed multiple of the PSD-weighted
data power in that bin, so the statistic of one track is

    S[j] = sum_alpha P[alpha, b(j, alpha)],
    b(j, alpha) = rint((f0[alpha] + sum_k c[j, k] U[alpha, k]) * T_SFT),

with the track rebuilt from the basis by the matrix product of Eq. (10) and the
bin width 1/T_SFT of Sec. II B.  A segment whose bin falls outside
[k_min, k_max] (or whose position is not finite) contributes nothing, as the
paper gives no contribution to segments it excludes (Sec. II B validity cut;
Sec. II D frequency cut-off).  Sec. II D keeps the best-scoring candidates of a
batch; the top-k here orders by (-S, template index).

Readings: rint is IEEE round-half-to-even; coefficients are FP32 and widened
exactly; the segment sum and everything else is FP64.  A position within
NEAR_TIE_BAND of a half-integer is flagged as a near tie (both neighbouring
bins are then acceptable from any implementation that rounds differently).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

NEAR_TIE_BAND = 1e-6


def track_positions(f0, U, coeffs, t_sft: float) -> np.ndarray:
    """x[j, alpha] = (f0[alpha] + sum_k c[j,k] U[alpha,k]) * T_SFT in bins (FP64)."""
    f0 = np.asarray(f0, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64).reshape(f0.size, -1)
    c = np.asarray(coeffs, dtype=np.float32).astype(np.float64)
    if c.ndim != 2 or c.shape[1] != U.shape[1]:
        raise ValueError("coeffs must be (n_tmpl, K)")
    freq = f0[None, :] + c @ U.T
    return freq * float(t_sft)


def chosen_bins(x: np.ndarray, n_bins: int, k_min: int = 0, k_max: int | None = None):
    """Nearest bin and validity: b = rint(x); valid iff x finite and k_min <= b <= k_max."""
    if k_max is None:
        k_max = n_bins - 1
    finite = np.isfinite(x)
    b = np.where(finite, np.rint(np.where(finite, x, 0.0)), 0.0)
    valid = finite & (b >= k_min) & (b <= k_max)
    return b.astype(np.int64), valid


def near_tie_mask(x: np.ndarray) -> np.ndarray:
    finite = np.isfinite(x)
    xs = np.where(finite, x, 0.0)
    return finite & (np.abs(xs - np.floor(xs) - 0.5) < NEAR_TIE_BAND)


def topk_order(stat: np.ndarray, top_k: int):
    """First top_k templates by key (-S, j); padded with (-inf, -1) past n_tmpl."""
    stat = np.asarray(stat, dtype=np.float64)
    n = stat.size
    order = np.lexsort((np.arange(n), -stat))[: min(top_k, n)]
    vals = np.full(top_k, -np.inf)
    idx = np.full(top_k, -1, dtype=np.int64)
    vals[: order.size] = stat[order]
    idx[: order.size] = order
    return vals, idx


def score_tracks(P, f0, U, coeffs, t_sft: float, top_k: int = 0, k_min: int = 0,
                 k_max: int | None = None, want_bins: bool = False, chunk: int = 65536):
    """Statistic, top-k, optional bins and the near-tie count for a coefficient batch.

    P      : (n_seg, n_bins) normalised power (any float dtype; widened to FP64)
    f0     : (n_seg,) offset track in Hz;  U : (n_seg, K) basis in Hz
    coeffs : (n_tmpl, K) FP32 coefficient vectors
    Returns a dict with ``stat`` (FP64), ``topk_val``, ``topk_idx``, ``n_near_tie``
    and, if requested, ``bins`` (int32, -1 where the segment does not contribute).
    """
    P = np.asarray(P, dtype=np.float64)
    n_seg, n_bins = P.shape
    coeffs = np.asarray(coeffs, dtype=np.float32)
    Um = np.asarray(U, dtype=np.float64).reshape(n_seg, -1)
    K = Um.shape[1]
    if coeffs.ndim != 2 or coeffs.shape[1] != K:
        raise ValueError("coeffs must be (n_tmpl, K)")
    n_tmpl = coeffs.shape[0]
    stat = np.zeros(n_tmpl)
    bins = np.empty((n_tmpl, n_seg), dtype=np.int32) if want_bins else None
    n_near = 0
    rows = np.arange(n_seg)[None, :]
    for s in range(0, n_tmpl, chunk):
        x = track_positions(f0, Um, coeffs[s:s + chunk], t_sft)
        b, valid = chosen_bins(x, n_bins, k_min, k_max)
        vals = np.where(valid, P[rows, np.where(valid, b, 0)], 0.0)
        stat[s:s + chunk] = vals.sum(axis=1)
        n_near += int(near_tie_mask(x).sum())
        if want_bins:
            bins[s:s + chunk] = np.where(valid, b, -1)
    vals, idx = topk_order(stat, top_k)
    out = dict(stat=stat, topk_val=vals, topk_idx=idx, n_near_tie=n_near)
    if want_bins:
        out["bins"] = bins
    return out


def _round_half_even(q: Fraction) -> int:
    return round(q)          # Fraction.__round__ rounds halves to even


def score_tracks_exact(P, f0, U, coeffs, t_sft: float, k_min: int = 0, k_max: int | None = None):
    """Brute force in exact rational arithmetic, for tiny inputs.

    Every FP64/FP32 input is converted exactly to a Fraction; the position,
    its rounding and the segment sum are exact, and the sum is rounded once.
    Returns (stat[n_tmpl] FP64, bins[n_tmpl, n_seg] with -1 for no contribution).
    """
    P = np.asarray(P, dtype=np.float64)
    n_seg, n_bins = P.shape
    if k_max is None:
        k_max = n_bins - 1
    f0 = [Fraction(float(v)) for v in np.asarray(f0, dtype=np.float64)]
    Um = np.asarray(U, dtype=np.float64).reshape(n_seg, -1)
    K = Um.shape[1]
    C = np.asarray(coeffs, dtype=np.float32)
    T = Fraction(float(t_sft))
    stat = np.zeros(C.shape[0])
    bins = np.full((C.shape[0], n_seg), -1, dtype=np.int64)
    for j in range(C.shape[0]):
        total = Fraction(0)
        for a in range(n_seg):
            f = f0[a]
            for k in range(K):
                f += Fraction(float(C[j, k])) * Fraction(float(Um[a, k]))
            b = _round_half_even(f * T)
            if k_min <= b <= k_max:
                bins[j, a] = b
                total += Fraction(float(P[a, b]))
        stat[j] = float(total)
    return stat, bins


def fsum_rows(P, bins) -> np.ndarray:
    """Correctly rounded segment sums for given bins (-1 = no contribution)."""
    P = np.asarray(P, dtype=np.float64)
    out = np.zeros(bins.shape[0])
    for j in range(bins.shape[0]):
        out[j] = math.fsum(P[a, b] for a, b in enumerate(bins[j]) if b >= 0)
    return out
