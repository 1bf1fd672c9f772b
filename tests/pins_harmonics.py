"""Checks that pin the multi-harmonic oracle (Sec. IV) to exact arithmetic.

* Exact rational brute force on tiny inputs: every harmonic's position
  r_h (f0 + sum_k c_k U_k) T is formed as a Fraction and rounded half to
  even, with ratios 1/2, 3/2 and 2 placing scaled positions exactly on half
  bins (a rounding of the unscaled bin first, or a scaling of f0 alone, gives
  different bins).
* The constant-track identity: with K = 0 and f0 = b / T every segment of
  harmonic h picks bin rint(r_h b), so S = sum_h sum_alpha P[alpha, rint(r_h b)].
* Additivity over harmonics: the statistic of a union of ratio sets is the
  sum of the statistics of its parts.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

RATIOS = (1.0, 0.5, 1.5, 2.0)


def _tiny(seed):
    g = np.random.default_rng(60 + seed)
    n_seg, n_bins, K, T = 4, 40, 2, 8.0
    P = g.uniform(0.0, 3.0, (n_seg, n_bins))
    f0 = g.integers(4, 12, n_seg) / T                       # x on whole bins before the coefficients
    U = g.choice([-1.0, -0.5, 0.5, 1.0], (n_seg, K)) / T
    C = g.choice([-3.0, -1.0, 0.0, 1.0, 3.0], (8, K)).astype(np.float32)
    C[0] = [1.0, 0.0]                                       # odd positions: r = 1/2, 3/2 land on exact halves
    return P, f0, U, C, T


def check_harmonics_exact(score_harmonics):
    for seed in range(4):
        P, f0, U, C, T = _tiny(seed)
        got = score_harmonics(P, f0, U, C, T, RATIOS)["stat"]
        n_seg, n_bins = P.shape
        for j in range(C.shape[0]):
            total = Fraction(0)
            for r in RATIOS:
                for a in range(n_seg):
                    pos = Fraction(float(f0[a]))
                    for k in range(U.shape[1]):
                        pos += Fraction(float(C[j, k])) * Fraction(float(U[a, k]))
                    b = round(Fraction(r) * pos * Fraction(T))         # exact, half to even
                    if 0 <= b < n_bins:
                        total += Fraction(float(P[a, b]))
            assert abs(float(got[j]) - float(total)) <= 1e-14 * max(1.0, float(total)), (seed, j)


def check_harmonics_constant_track(score_harmonics):
    g = np.random.default_rng(61)
    n_seg, n_bins, T = 5, 64, 100.0
    P = g.exponential(size=(n_seg, n_bins))
    for b in (3, 10, 21, 40):
        f0 = np.full(n_seg, b / T)
        got = score_harmonics(P, f0, np.zeros((n_seg, 0)), np.zeros((2, 0), np.float32), T, RATIOS)["stat"]
        want = 0.0
        for r in RATIOS:
            bh = round(Fraction(r) * b)
            if bh < n_bins:
                want += P[:, bh].sum()
        assert np.allclose(got, want, rtol=1e-14, atol=0), (b, got, want)


def check_harmonics_additive(score_harmonics):
    g = np.random.default_rng(62)
    n_seg, n_bins, K, T = 9, 300, 3, 1e3
    P = g.exponential(size=(n_seg, n_bins))
    f0 = g.uniform(0.05, 0.15, n_seg)
    U = g.standard_normal((n_seg, K)) * 0.02
    C = g.uniform(-1, 1, (50, K)).astype(np.float32)
    a = score_harmonics(P, f0, U, C, T, (1.0, 0.5))["stat"]
    b = score_harmonics(P, f0, U, C, T, (1.5,))["stat"]
    ab = score_harmonics(P, f0, U, C, T, (1.0, 0.5, 1.5))["stat"]
    assert np.allclose(ab, a + b, rtol=1e-13, atol=0)
    one = score_harmonics(P, f0, U, C, T, (1.0,))
    assert one["topk_idx"].size == 0
    assert np.all(np.asarray(one["stat"]) > 0)
