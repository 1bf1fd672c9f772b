"""Oracle: the linear-chirp semi-coherent statistic (test infrastructure only).

Sec. II B models the signal in each SFT segment as a chirping sinusoid with
local frequency f_alpha and derivative fdot_alpha (Eqs. (4)-(5)), maximises
the inner product over amplitude and phase (Eq. (7)), and evaluates it in the
SFT domain over the 2P + 1 bins around the signal (P = 100); a segment whose
second derivative breaks the linear approximation (fddot T^3 / 6 > 1) and,
in the search of Sec. II D, frequencies below 10^-3.5 Hz or derivatives below
1e-13 Hz/s contribute nothing.  The local parameters come from the track
rebuilt from the basis (Eq. (10)), fdot numerically (Sec. II C).

Definitions written out here (the readings are listed with each function):

* whitened complex SFT of the data, Z[alpha, k] = X_k / sqrt(sum w^2 S(f_k) / (2 dt)),
  X_k the DFT of the Hann-windowed segment (|Z|^2 is the power P of build_sfts);
* template SFT of the unit linear chirp exp(i[2 pi f (t - t_a) + pi fdot (t - t_a)^2]),
  windowed the same way, in the continuum limit:
      H_k = (-1)^k R(f T - k, fdot T^2),  R(d, b) = int_{-1/2}^{1/2} cos^2(pi u) exp(2 pi i d u + i pi b u^2) du
  (the common factor T/dt is dropped; (-1)^k because the DFT's time origin is
  the segment's start, the chirp's its midpoint);
* per segment, with k0 = rint(f T) inside the row (else the segment
  contributes nothing, as a position outside the row does in the nearest-bin
  statistic) and the bins k0 - P..k0 + P inside the row,
      S_alpha = |sum_k conj(Z_k) H_k / sqrt(S_k)|^2 / sum_k |H_k|^2 / S_k ,
  which is (max over phase of <d|h>)^2 / <h|h> up to the constant 2 sum w^2 / N
  (= 3/4 for the Hann window), dropped so that with P = 0 the statistic is the
  nearest-bin power P[alpha, k0] whatever the template; bins whose PSD is not
  positive and finite take no part;
* S = sum over valid segments of S_alpha.
"""
from __future__ import annotations

import numpy as np

from .sft import hann_periodic, segments, normaliser
from .score import track_positions

P_HALF = 100                   # 2P + 1 = 201 bins
F_MIN = 10.0 ** -3.5           # Hz
FDOT_MIN = 1e-13               # Hz / s


def build_sfts_complex(x, dt: float, n_sft: int, psd) -> np.ndarray:
    """Whitened complex SFTs Z[alpha, k] (complex128), k = 0..n_sft/2."""
    seg = segments(np.asarray(x, dtype=np.float64), n_sft)
    w = hann_periodic(n_sft)
    X = np.fft.rfft(seg * w[None, :], axis=1)
    psd = np.asarray(psd, dtype=np.float64)
    ok = np.isfinite(psd) & (psd > 0)
    norm = normaliser(w, np.where(ok, psd, 1.0), dt)
    Z = X / np.sqrt(norm)[None, :]
    Z[:, ~ok] = 0.0
    return Z


def inverse_sqrt_psd(psd) -> np.ndarray:
    """1 / sqrt(S_k), 0 where the PSD is not positive and finite."""
    psd = np.asarray(psd, dtype=np.float64)
    ok = np.isfinite(psd) & (psd > 0)
    return np.where(ok, 1.0 / np.sqrt(np.where(ok, psd, 1.0)), 0.0)


def track_derivatives(f, t_sft: float):
    """fdot and fddot of tracks sampled at the segment midpoints (rows of f).

    Reading: second-order finite differences on the segment grid (spacing
    T_SFT): central in the interior, second-order one-sided at both ends for
    fdot (all exact for quadratic tracks); fddot from second differences, the
    end segments taking their neighbour's value."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[-1]
    T = float(t_sft)
    fd = np.empty_like(f)
    fdd = np.empty_like(f)
    if n < 3:
        fd[...] = 0.0 if n == 1 else ((f[..., 1:2] - f[..., 0:1]) / T)
        fdd[...] = 0.0
        return fd, fdd
    fd[..., 1:-1] = (f[..., 2:] - f[..., :-2]) / (2.0 * T)
    fd[..., 0] = (-3.0 * f[..., 0] + 4.0 * f[..., 1] - f[..., 2]) / (2.0 * T)
    fd[..., -1] = (3.0 * f[..., -1] - 4.0 * f[..., -2] + f[..., -3]) / (2.0 * T)
    fdd[..., 1:-1] = (f[..., 2:] - 2.0 * f[..., 1:-1] + f[..., :-2]) / (T * T)
    fdd[..., 0] = fdd[..., 1]
    fdd[..., -1] = fdd[..., -2]
    return fd, fdd


def _gauss_grid(cycles: float, nodes: int = 16):
    """Gauss-Legendre nodes and weights on [-1/2, 1/2] with one panel per
    half cycle of the fastest oscillation (16 nodes each: exact to rounding)."""
    panels = int(np.ceil(2.0 * cycles)) + 2
    x, w = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(-0.5, 0.5, panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    u = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    wt = (half[:, None] * w[None, :]).ravel()
    return u, wt


def chirp_template_bins(delta0: float, beta: float, p_half: int) -> np.ndarray:
    """R(delta0 - m, beta) for m = -p_half..p_half (complex128), by quadrature
    of the defining integral with the Hann window cos^2(pi u)."""
    m = np.arange(-p_half, p_half + 1)
    u, wt = _gauss_grid(abs(delta0) + p_half + abs(beta) + 1.0)
    g = wt * np.cos(np.pi * u) ** 2 * np.exp(1j * (2.0 * np.pi * delta0 * u + np.pi * beta * u * u))
    return np.exp(-2j * np.pi * np.outer(m, u)) @ g


def segment_statistic(Z_row, isq, f: float, fdot: float, t_sft: float, p_half: int) -> float:
    """S_alpha of one segment (FP64) for local frequency f and derivative fdot."""
    n_bins = Z_row.shape[0]
    x = f * t_sft
    if not np.isfinite(x) or not (-0.5 <= x < n_bins - 0.5):
        return 0.0                          # the central bin is outside the row
    k0 = int(np.rint(x))
    if not 0 <= k0 < n_bins:
        return 0.0
    m = np.arange(-p_half, p_half + 1)
    k = k0 + m
    inside = (k >= 0) & (k < n_bins)
    H = chirp_template_bins(x - k0, fdot * t_sft * t_sft, p_half)
    H = H * np.where(k % 2 == 0, 1.0, -1.0)
    kk = np.where(inside, k, 0)
    Hw = np.where(inside, H * isq[kk], 0.0)
    Zk = np.where(inside, Z_row[kk], 0.0)
    den = float(np.sum(np.abs(Hw) ** 2))
    if den == 0.0:
        return 0.0
    return float(np.abs(np.sum(np.conj(Zk) * Hw)) ** 2 / den)


def segment_valid(f, fdot, fddot, t_sft: float, f_min: float = F_MIN, fdot_min: float = FDOT_MIN):
    """Segments that contribute: the linear approximation holds (|fddot| T^3 / 6 <= 1)
    and f >= f_min, fdot >= fdot_min (Sec. II D cut-offs; pass -inf to disable)."""
    T = float(t_sft)
    return (np.abs(fddot) * T ** 3 / 6.0 <= 1.0) & (f >= f_min) & (fdot >= fdot_min)


def score_chirp(Z, isq, f0, U, coeffs, t_sft: float, p_half: int = P_HALF, f_min: float = F_MIN,
                fdot_min: float = FDOT_MIN, top_k: int = 0):
    """Linear-chirp statistic of a coefficient batch (slow; small inputs).

    Z: (n_seg, n_bins) whitened complex SFTs; isq: (n_bins,) 1/sqrt(S).
    Returns dict(stat FP64[n_tmpl], per_segment [n_tmpl, n_seg], valid, topk_val, topk_idx)."""
    from .score import topk_order
    Z = np.asarray(Z)
    n_seg = Z.shape[0]
    f = track_positions(f0, U, coeffs, 1.0)                 # Hz: positions at T = 1
    fd, fdd = track_derivatives(f, t_sft)
    valid = segment_valid(f, fd, fdd, t_sft, f_min, fdot_min)
    per = np.zeros(f.shape)
    for j in range(f.shape[0]):
        for a in range(n_seg):
            if valid[j, a]:
                per[j, a] = segment_statistic(Z[a], isq, f[j, a], fd[j, a], t_sft, p_half)
    stat = per.sum(axis=1)
    vals, idx = topk_order(stat, top_k)
    return dict(stat=stat, per_segment=per, valid=valid, topk_val=vals, topk_idx=idx)
