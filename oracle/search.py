"""Oracle: population search over basis coefficients (test infrastructure only).

Sec. II D maximises the statistic over the coefficients with a population of
walkers:

* seeding -- draw candidates uniformly in the prior box; move each track so
  that its initial frequency is a value drawn uniformly in a given range and
  project the moved track back onto the basis; score every candidate and keep
  the best ones as the walkers;
* differential evolution in track space, Eq. (11) -- every walker's track gets
  the trial  f_trial = f + F (f_r1 - f_r2)  with two other walkers r1 != r2
  and a weight F drawn in [0.3, 1.5], with no crossover; a trial that scores
  higher and lies inside the prior is projected back to coefficients with the
  pseudo-inverse of the basis and replaces the walker.

The gradient (Adam) half of each iteration is not reproduced: the nearest-bin
statistic is piecewise constant in the coefficients, so its gradient is zero
almost everywhere.

Readings (the paper is silent on them): random numbers (candidate draws,
initial frequencies, r1, r2, F) are inputs, drawn by the caller; a walker is
stored as an FP32 coefficient vector, the representation the scorer takes, so
a trial is projected and rounded to FP32 before it is scored (in exact
arithmetic the trial track lies in the span of the basis, so scoring the track
or its projection is the same); the prior check is on those FP32 coefficients
against the box, bounds included; "better" is strictly greater; the initial
frequency of a track is its value in the first segment, and moving the track
means adding one constant to every segment before the projection.
"""
from __future__ import annotations

import numpy as np

from .score import score_tracks, topk_order


def tracks_of(f0, U, coeffs) -> np.ndarray:
    """f[j, alpha] = f0[alpha] + sum_k c[j, k] U[alpha, k] (Hz, FP64) -- Eq. (10)."""
    U = np.asarray(U, dtype=np.float64)
    c = np.asarray(coeffs, dtype=np.float32).astype(np.float64)
    return np.asarray(f0, dtype=np.float64)[None, :] + c @ U.T


def project(f0, U, tracks) -> np.ndarray:
    """Coefficients of tracks through the pseudo-inverse of the basis (FP64)."""
    U = np.asarray(U, dtype=np.float64)
    return (np.asarray(tracks, dtype=np.float64) - np.asarray(f0, dtype=np.float64)[None, :]) @ np.linalg.pinv(U).T


def seed_candidates(f0, U, draws, f_init) -> np.ndarray:
    """Candidates whose first-segment frequency is moved to f_init, projected
    back onto the basis and stored as FP32."""
    f = tracks_of(f0, U, draws)
    moved = f + (np.asarray(f_init, dtype=np.float64) - f[:, 0])[:, None]
    return project(f0, U, moved).astype(np.float32)


def seed_population(P, f0, U, draws, f_init, t_sft: float, n_keep: int, k_min: int = 0, k_max=None):
    """Score the seeded candidates and keep the n_keep best by (-S, index).

    Returns (coeffs FP32[n_keep, K], stat FP64[n_keep], idx[n_keep] into the candidates)."""
    cand = seed_candidates(f0, U, draws, f_init)
    res = score_tracks(P, f0, U, cand, t_sft, 0, k_min, k_max)
    vals, idx = topk_order(res["stat"], n_keep)
    return cand[idx], vals, idx


def in_prior(coeffs, box_lo, box_hi) -> np.ndarray:
    c = np.asarray(coeffs, dtype=np.float32).astype(np.float64)
    return np.all((c >= np.asarray(box_lo)[None, :]) & (c <= np.asarray(box_hi)[None, :]), axis=1)


def de_trials(f0, U, coeffs, r1, r2, F) -> np.ndarray:
    """Eq. (11) in track space, projected back and stored as FP32."""
    f = tracks_of(f0, U, coeffs)
    r1 = np.asarray(r1, dtype=np.int64)
    r2 = np.asarray(r2, dtype=np.int64)
    trial = f + np.asarray(F, dtype=np.float64)[:, None] * (f[r1] - f[r2])
    return project(f0, U, trial).astype(np.float32)


def de_generation(P, f0, U, box_lo, box_hi, coeffs, stat, r1, r2, F, t_sft: float, k_min: int = 0, k_max=None):
    """One differential-evolution generation over the whole population.

    coeffs FP32[n, K], stat[n] (the walkers' current statistics); r1, r2 int[n]
    (each differs from the walker's own index and from each other); F[n].
    Returns dict(coeffs, stat, accepted, trial, trial_stat, in_prior)."""
    n = np.asarray(coeffs).shape[0]
    r1 = np.asarray(r1, dtype=np.int64)
    r2 = np.asarray(r2, dtype=np.int64)
    own = np.arange(n)
    if np.any((r1 == own) | (r2 == own) | (r1 == r2)):
        raise ValueError("r1, r2 and the walker must be three different walkers")
    trial = de_trials(f0, U, coeffs, r1, r2, F)
    trial_stat = score_tracks(P, f0, U, trial, t_sft, 0, k_min, k_max)["stat"]
    inside = in_prior(trial, box_lo, box_hi)
    accepted = inside & (trial_stat > np.asarray(stat, dtype=np.float64))
    new_c = np.where(accepted[:, None], trial, np.asarray(coeffs, dtype=np.float32))
    new_s = np.where(accepted, trial_stat, np.asarray(stat, dtype=np.float64))
    return dict(coeffs=new_c, stat=new_s, accepted=accepted, trial=trial, trial_stat=trial_stat, in_prior=inside)


# ------------------------------------------------------- progressive durations
# Sec. II D searches data of growing duration with the plunge at the end of
# each: the one-year basis is shifted by a whole number of segments, so that a
# chain on the first n segments uses the basis rows of the last n segments;
# each duration's best statistic is normalised by the mean and standard
# deviation of the same search on noise-only data.  Readings: the standard
# deviation is the sample one (denominator R - 1 over R realisations); the
# best walker is the first by (-S, index) with NaN last.


def shifted_basis(f0, U, n: int):
    """Basis rows of the last n segments (the basis shifted by len(f0) - n segments)."""
    f0 = np.asarray(f0, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    N = f0.size
    if not 1 <= n <= N:
        raise ValueError("duration outside the basis")
    return f0[N - n:], U[N - n:]


def noise_moments(best) -> tuple:
    """Mean and sample standard deviation over realisations (axis 0) of each chain's best statistic."""
    b = np.asarray(best, dtype=np.float64)
    return b.mean(axis=0), b.std(axis=0, ddof=1)


def normalised(stat, mean, sd):
    return (np.asarray(stat, dtype=np.float64) - np.asarray(mean)) / np.asarray(sd)


def best_walker(stat) -> int:
    s = np.asarray(stat, dtype=np.float64)
    key = np.where(np.isnan(s), -np.inf, s)
    rank_nan = np.isnan(s).astype(np.int64)
    return int(np.lexsort((np.arange(s.size), -key, rank_nan))[0])
