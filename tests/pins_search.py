"""Checks that pin the search oracle (Sec. II D, Eq. (11)) to closed forms.

Each check takes the function under test, so the same checks run against the
oracle (they must pass) and against planted mistakes (one must fail; see
test_oracle_mutants.py).

* The trial of Eq. (11) is formed in track space and projected back with the
  pseudo-inverse of the basis.  For any basis of full column rank the
  projection inverts the reconstruction, so the trial's coefficients are
  c + F (c_r1 - c_r2) exactly in real arithmetic: checked with a basis that
  is not orthonormal (so that a transpose in place of the pseudo-inverse
  fails) to within the rounding of the FP32 result.
* Seeding moves a track by a constant so that its first-segment frequency is
  the drawn one: with a basis that contains the constant direction the moved
  track's first frequency equals the draw; in general the coefficients move by
  (f_init - f[0]) pinv(U) 1.
* Acceptance: a statistic that is linear in one coefficient (bin = segment's
  power index) makes every trial's statistic known in closed form; a trial is
  accepted exactly when it is inside the box (bounds included) and strictly
  better.
* Keeping the best seeds: the first n_keep by (-S, index) of a full sort.
"""
from __future__ import annotations

import numpy as np


def _basis(g, n_seg, K, constant=False):
    U = g.standard_normal((n_seg, K))
    if constant:
        U[:, 0] = 1.0
    U[:, -1] *= 3.0                      # not orthonormal: pinv(U) != U.T
    return U


def check_de_trial_closed_form(de_trials):
    g = np.random.default_rng(51)
    for K in (1, 3, 8):
        n_seg, n = 17, 40
        U = _basis(g, n_seg, K)
        f0 = g.uniform(1e-3, 2e-3, n_seg)
        c = g.uniform(-2, 2, (n, K)).astype(np.float32)
        r1 = (np.arange(n) + 1 + g.integers(0, n - 2, n)) % n
        r2 = r1.copy()
        for i in range(n):
            while r2[i] in (i, r1[i]):
                r2[i] = g.integers(0, n)
        F = g.uniform(0.3, 1.5, n)
        got = np.asarray(de_trials(f0, U, c, r1, r2, F))
        want = c.astype(np.float64) + F[:, None] * (c[r1].astype(np.float64) - c[r2].astype(np.float64))
        assert got.dtype == np.float32 and got.shape == (n, K)
        scale = np.abs(c).max() * (1 + 2 * 1.5)
        assert np.all(np.abs(got - want) <= 2.0 ** -23 * np.abs(want) + 1e-12 * scale), np.abs(got - want).max()


def check_seed_closed_form(seed_candidates):
    g = np.random.default_rng(52)
    n_seg, n, K = 23, 30, 4
    f0 = g.uniform(1e-3, 2e-3, n_seg)
    draws = g.uniform(-1e-4, 1e-4, (n, K)).astype(np.float32)
    f_init = g.uniform(5e-4, 1e-2, n)
    # a basis holding the constant direction: the first frequency becomes the draw
    U = _basis(g, n_seg, K, constant=True)
    got = np.asarray(seed_candidates(f0, U, draws, f_init))
    assert got.dtype == np.float32
    first = f0[0] + got.astype(np.float64) @ U[0]
    assert np.all(np.abs(first - f_init) <= 1e-6 * f_init), np.abs(first - f_init).max()
    # in general the coefficients move by (f_init - f[0]) pinv(U) 1
    U = _basis(g, n_seg, K)
    got = np.asarray(seed_candidates(f0, U, draws, f_init)).astype(np.float64)
    f_first = f0[0] + draws.astype(np.float64) @ U[0]
    step = np.linalg.lstsq(U, np.ones(n_seg), rcond=None)[0]
    want = draws.astype(np.float64) + (f_init - f_first)[:, None] * step[None, :]
    assert np.all(np.abs(got - want) <= 2.0 ** -23 * np.abs(want) + 1e-12), np.abs(got - want).max()


def check_de_acceptance(de_generation):
    """K = 1, U = 1/T per segment: the track sits at bin f0 T + c in every
    segment, and P[a, b] = b, so S(c) = sum_a rint(f0_a T + c) is known."""
    n_seg, n_bins, T = 5, 200, 10.0
    P = np.tile(np.arange(n_bins, dtype=np.float64), (n_seg, 1))
    f0 = np.array([5.0, 6.0, 7.0, 8.0, 9.0]) / T
    U = np.full((n_seg, 1), 1.0 / T)
    c = np.array([[10.0], [20.0], [30.0], [40.0], [50.0], [60.0]], dtype=np.float32)

    def S(v):
        return float(sum(np.rint(f0[a] * T + v) for a in range(n_seg)))

    stat = np.array([S(v) for v in c[:, 0]])
    box_lo, box_hi = np.array([0.0]), np.array([70.0])
    # walker 0: 10 + 1.0 (60 - 20) = 50: better, inside -> accepted
    # walker 1: 20 + 0.5 (10 - 30) = 10: worse -> kept
    # walker 2: 30 + 1.0 (60 - 20) = 70: on the upper bound, better -> accepted
    # walker 3: 40 + 1.5 (60 - 10) = 115: better, outside the box -> kept
    # walker 4: 50 + 1e-3 (40 - 20) = 50.02: the same bins, an equal S -> kept
    # walker 5: 60 + 0.3 (10 - 50) = 48: worse -> kept
    r1 = np.array([5, 0, 5, 5, 3, 0])
    r2 = np.array([1, 2, 1, 0, 1, 4])
    F = np.array([1.0, 0.5, 1.0, 1.5, 1e-3, 0.3])
    out = de_generation(P, f0, U, box_lo, box_hi, c, stat, r1, r2, F, T)
    trial = np.asarray(out["trial"], dtype=np.float64)[:, 0]
    assert np.allclose(trial, [50.0, 10.0, 70.0, 115.0, 50.02, 48.0], rtol=1e-6)
    assert list(np.asarray(out["accepted"])) == [True, False, True, False, False, False]
    want_c = np.where([True, False, True, False, False, False], trial, c[:, 0])
    assert np.allclose(np.asarray(out["coeffs"])[:, 0], want_c, rtol=1e-6)
    assert np.allclose(out["stat"], [S(v) for v in want_c])
    for j, v in enumerate(trial):
        assert out["trial_stat"][j] == S(np.float32(v))


def check_seed_keeps_best(seed_population):
    g = np.random.default_rng(53)
    n_seg, n_bins, T, K, n = 6, 300, 100.0, 2, 64
    P = np.round(g.exponential(size=(n_seg, n_bins)), 1)
    f0 = g.uniform(0.5, 2.5, n_seg)
    U = g.standard_normal((n_seg, K)) * 0.2
    draws = g.uniform(-1, 1, (n, K)).astype(np.float32)
    draws[10:14] = draws[3]                        # exact ties: index order decides
    f_init = np.full(n, f0[0])
    coeffs, stat, idx = seed_population(P, f0, U, draws, f_init, T, 20)
    from oracle.search import seed_candidates
    from oracle.score import score_tracks
    cand = seed_candidates(f0, U, draws, f_init)
    full = score_tracks(P, f0, U, cand, T, 0)["stat"]
    order = sorted(range(n), key=lambda j: (-full[j], j))[:20]
    assert list(idx) == order
    assert np.array_equal(np.asarray(coeffs), cand[order])
    assert np.array_equal(np.asarray(stat), full[order])


def check_shifted_basis(shifted_basis):
    """A full-rank basis of tracks that end at the plunge: the last n rows,
    with a track's own coefficients, rebuild that track's last n values."""
    g = np.random.default_rng(54)
    N, n_train = 40, 12
    F = np.cumsum(g.uniform(0, 1e-4, (n_train, N)), axis=1) + g.uniform(1e-3, 5e-3, (n_train, 1))
    f0 = F.mean(axis=0)
    X = F - f0
    _, _, vt = np.linalg.svd(X, full_matrices=False)
    U = vt[:n_train].T
    c = X @ U
    for n in (1, 7, 25, N):
        fs, Us = shifted_basis(f0, U, n)
        assert fs.shape == (n,) and Us.shape == (n, U.shape[1])
        assert np.allclose(fs[None, :] + c @ Us.T, F[:, N - n:], rtol=0, atol=1e-15)


def check_noise_moments(noise_moments):
    import statistics
    g = np.random.default_rng(55)
    best = g.normal(100.0, 3.0, (6, 5))
    best[:, 2] = 7.0                                   # no spread
    best[:, 3] = [0.0, 2.0, 0.0, 2.0, 0.0, 2.0]
    mean, sd = noise_moments(best)
    for c in range(best.shape[1]):
        col = [float(v) for v in best[:, c]]
        assert abs(mean[c] - statistics.fmean(col)) <= 1e-12 * abs(mean[c]) + 1e-15
        assert abs(sd[c] - statistics.stdev(col)) <= 1e-12 * max(sd[c], 1.0)
    assert sd[2] == 0.0 and abs(sd[3] - np.sqrt(1.2)) <= 1e-15


def check_best_walker(best_walker):
    assert best_walker([1.0, 3.0, 2.0, 3.0]) == 1                 # ties: lower index
    assert best_walker([np.nan, -5.0, -7.0]) == 1                  # NaN ranks last
    assert best_walker([np.nan, np.nan]) == 0
    assert best_walker([-np.inf, -1e30]) == 1
