"""Checks that pin the oracle to the paper and to mathematics, not to itself.

Each check takes the implementation under test as an argument, so the same
checks run against the oracle (they must pass) and against oracle variants with
a planted mistake (at least one must fail; see test_oracle_mutants.py).

What pins what:
* SFT power (Sec. II B, Eq. (7)): a direct O(N^2) DFT with the window's closed
  sum  sum_n w_n^2 = 3N/8;  Parseval per segment;  the closed-form response of a
  Hann-windowed sinusoid (finite geometric sums);  the Exp(1) law of noise-only
  power and the Gamma(N_seg, 1) law of the segment sum.
* Basis (Sec. II C, Eqs. (9)-(10)): orthonormality;  Eckart-Young residual;
  exact reconstruction at full rank;  agreement with the eigenvectors of the
  Gram matrix;  a rank-one family whose projections and quantiles are known in
  closed form;  the sign rule.
* Statistic (Eq. (6), nearest-bin limit; Eq. (10)): exact rational brute force
  including constructed half-bin ties and out-of-range bins;  the column-sum
  identity of a constant track;  template permutation;  top-k against a full
  sort of (-S, j) tuples.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import stats

# ----------------------------------------------------------------------------- SFT


def _direct_dft(seg: np.ndarray) -> np.ndarray:
    """X_b = sum_n seg_n exp(-2 pi i b n / N) for b = 0..N/2, by the definition."""
    n = seg.size
    out = np.empty(n // 2 + 1, dtype=np.complex128)
    for b in range(n // 2 + 1):
        acc = 0j
        for k in range(n):
            ang = -2.0 * math.pi * ((b * k) % n) / n
            acc += seg[k] * complex(math.cos(ang), math.sin(ang))
        out[b] = acc
    return out


def check_sft_bruteforce(build_sfts):
    g = np.random.default_rng(11)
    for n_sft in (8, 12, 30, 60):
        dt = 0.5 + g.uniform()
        n_seg = 3
        x = g.standard_normal(n_seg * n_sft + n_sft // 3)       # ragged tail is dropped
        n_bins = n_sft // 2 + 1
        psd = g.uniform(0.5, 3.0, n_bins)
        psd[1] = 0.0
        psd[-2 if n_bins > 3 else 0] = np.inf
        P = np.asarray(build_sfts(x, dt, n_sft, psd))
        assert P.shape == (n_seg, n_bins)
        window = np.array([math.sin(math.pi * k / n_sft) ** 2 for k in range(n_sft)])
        sum_w2 = 3.0 * n_sft / 8.0
        for a in range(n_seg):
            X = _direct_dft(window * x[a * n_sft:(a + 1) * n_sft])
            for b in range(n_bins):
                if not (np.isfinite(psd[b]) and psd[b] > 0):
                    assert P[a, b] == 0.0
                    continue
                want = abs(X[b]) ** 2 / (sum_w2 * psd[b] / (2.0 * dt))
                assert abs(P[a, b] - want) <= 1e-12 * max(1.0, want), (n_sft, a, b)


def check_sft_parseval(build_sfts):
    g = np.random.default_rng(12)
    for n_sft in (16, 8640):
        dt = 10.0
        n_seg = 4
        x = g.standard_normal(n_seg * n_sft) * 3.0 + 0.7
        level = 2.0 * dt                      # makes P = |X_b|^2 / sum w^2
        P = np.asarray(build_sfts(x, dt, n_sft, np.full(n_sft // 2 + 1, level)))
        absx2 = P * (3.0 * n_sft / 8.0)
        for a in range(n_seg):
            seg = x[a * n_sft:(a + 1) * n_sft] * np.sin(np.pi * np.arange(n_sft) / n_sft) ** 2
            lhs = float(np.sum(seg * seg))
            rhs = (absx2[a, 0] + 2.0 * absx2[a, 1:-1].sum() + absx2[a, -1]) / n_sft
            assert abs(lhs - rhs) <= 1e-12 * lhs


def _geom(mu: float, n: int) -> complex:
    """G(mu) = sum_{k<n} exp(2 pi i mu k / n) in closed form."""
    if abs(mu - round(mu)) < 1e-15 and round(mu) % n == 0:
        return complex(n)
    num = 1.0 - complex(math.cos(2 * math.pi * mu), math.sin(2 * math.pi * mu))
    den = 1.0 - complex(math.cos(2 * math.pi * mu / n), math.sin(2 * math.pi * mu / n))
    return num / den


def _hann_response(nu: float, n: int) -> complex:
    """W(nu) = sum_k sin^2(pi k/n) exp(2 pi i nu k/n) = G(nu)/2 - G(nu+1)/4 - G(nu-1)/4."""
    return 0.5 * _geom(nu, n) - 0.25 * _geom(nu + 1, n) - 0.25 * _geom(nu - 1, n)


def check_sft_sinusoid(build_sfts):
    """A noiseless sinusoid at b0 + delta lands in bin b0 with the closed-form power."""
    n_sft, dt, n_seg = 8640, 10.0, 5
    psd_level = 20.0
    g = np.random.default_rng(13)
    for b0, delta in ((37, 0.3), (1500, -0.45), (4000, 0.05), (2, 0.2)):
        amp, phi = 0.8 + g.uniform(), g.uniform(0, 2 * math.pi)
        f = (b0 + delta) / (n_sft * dt)
        t = np.arange(n_seg * n_sft) * dt
        x = amp * np.cos(2 * math.pi * f * t + phi)
        P = np.asarray(build_sfts(x, dt, n_sft, np.full(n_sft // 2 + 1, psd_level)))
        norm = (3.0 * n_sft / 8.0) * psd_level / (2.0 * dt)
        for a in range(n_seg):
            assert int(np.argmax(P[a])) == b0
            phase = phi + 2 * math.pi * (b0 + delta) * a            # phase at segment start
            e = complex(math.cos(phase), math.sin(phase))
            X = 0.5 * amp * e * _hann_response(delta, n_sft) \
                + 0.5 * amp * e.conjugate() * _hann_response(-2 * b0 - delta, n_sft)
            want = abs(X) ** 2 / norm
            assert abs(P[a, b0] - want) <= 1e-10 * want, (b0, a, P[a, b0], want)


def check_sft_noise_law(build_sfts, score_tracks=None):
    """White noise: per-bin power ~ Exp(1); a constant-bin track sum ~ Gamma(N_seg, 1)."""
    n_sft, dt, n_seg, sigma = 8640, 10.0, 30, 1.0
    level = 2.0 * sigma ** 2 * dt
    samples = []
    inner = []
    for seed in range(2):
        g = np.random.default_rng(100 + seed)
        x = sigma * g.standard_normal(n_seg * n_sft)
        P = np.asarray(build_sfts(x, dt, n_sft, np.full(n_sft // 2 + 1, level)))
        inner.append(P[:, 2:n_sft // 2 - 1].ravel())
        cols = np.arange(2, n_sft // 2 - 1, 3)        # >= 3 bins apart: independent
        if score_tracks is None:
            samples.append(P[:, cols].sum(axis=0))
        else:
            t_sft = n_sft * dt
            f0 = np.zeros(n_seg)
            U = np.full((n_seg, 1), 1.0 / math.sqrt(n_seg))
            c = (cols / t_sft * math.sqrt(n_seg)).astype(np.float32)
            # FP32 coefficients must still round to the intended bin
            got = score_tracks(P, f0, U, c[:, None], t_sft, 0)["stat"]
            samples.append(np.asarray(got))
    inner = np.concatenate(inner)
    assert abs(inner.mean() - 1.0) < 5e-3 and abs(inner.var() - 1.0) < 2e-2
    s = np.concatenate(samples)
    assert abs(s.mean() - n_seg) < 4.0 * math.sqrt(n_seg / s.size)
    assert stats.kstest(s, stats.gamma(n_seg).cdf).pvalue > 1e-3


# ----------------------------------------------------------------------------- basis


def _chirp_tracks(n_train, n_seg, seed, t_sft=86400.0 * 7):
    g = np.random.default_rng(seed)
    t = (np.arange(n_seg) + 0.5) * t_sft
    f0 = g.uniform(2e-3, 1e-2, n_train)
    tau = g.uniform(3e7, 1.5e8, n_train)
    return f0[:, None] * (1.0 - t[None, :] / tau[:, None]) ** -0.375


def check_basis_identities(build_basis):
    F = _chirp_tracks(400, 40, 21)
    K = 6
    f0, U, sv, lo, hi = (np.asarray(v) for v in build_basis(F, K))
    assert U.shape == (40, K) and sv.shape == (K,) and f0.shape == (40,)
    # f0 is the centre of the training set: centred columns sum to zero
    X = F - f0[None, :]
    assert np.all(np.abs(X.sum(axis=0)) <= 1e-9 * np.abs(F).sum(axis=0))
    assert np.abs(U.T @ U - np.eye(K)).max() < 1e-13
    # Eckart-Young: the residual energy is what the kept singular values leave
    resid = np.linalg.norm(X - X @ U @ U.T) ** 2
    total = np.linalg.norm(X) ** 2
    assert abs(resid - (total - float(np.sum(sv ** 2)))) <= 1e-9 * total
    assert np.all(np.diff(sv) <= 0)
    # Gram-matrix eigenvectors span the same leading directions
    evals, evecs = np.linalg.eigh(X.T @ X)
    evals, evecs = evals[::-1], evecs[:, ::-1]
    for k in range(K):
        if sv[k] / sv[0] > 1e-6:
            assert abs(abs(float(U[:, k] @ evecs[:, k])) - 1.0) < 1e-8
            assert abs(sv[k] ** 2 - evals[k]) <= 1e-8 * evals[0]
    # sign rule: largest-magnitude entry of each column is positive
    for k in range(K):
        assert U[int(np.argmax(np.abs(U[:, k]))), k] > 0
    assert np.all(lo < hi)


def check_basis_full_rank(build_basis):
    F = _chirp_tracks(60, 12, 22)
    f0, U, sv, lo, hi = (np.asarray(v) for v in build_basis(F, 12))
    X = F - f0[None, :]
    assert np.abs(X @ U @ U.T - X).max() <= 1e-12 * np.abs(X).max()


def check_basis_rank_one(build_basis):
    """tracks_i = m + a_i u with a_i = i - (n-1)/2: projections and quantiles in closed form."""
    n, n_seg = 201, 16
    g = np.random.default_rng(23)
    m = g.uniform(1e-3, 2e-3, n_seg)
    u = g.standard_normal(n_seg)
    u /= np.linalg.norm(u)
    a = np.arange(n) - (n - 1) / 2.0
    F = m[None, :] + a[:, None] * u[None, :]
    f0, U, sv, lo, hi = (np.asarray(v) for v in build_basis(F, 1))
    assert np.abs(f0 - m).max() < 1e-12
    sgn = 1.0 if u[int(np.argmax(np.abs(u)))] > 0 else -1.0
    assert np.abs(U[:, 0] - sgn * u).max() < 1e-12
    assert abs(sv[0] - math.sqrt(float(np.sum(a * a)))) < 1e-9 * sv[0]
    # projections are sgn * a_i, an arithmetic sequence: the q-quantile is
    # -(n-1)/2 + q (n-1) with linear interpolation between order statistics
    want_lo = -(n - 1) / 2.0 + 0.00135 * (n - 1)
    want_hi = -(n - 1) / 2.0 + 0.99865 * (n - 1)
    assert abs(lo[0] - want_lo) < 1e-9 and abs(hi[0] - want_hi) < 1e-9


def check_basis_low_rank_recovery(build_basis):
    """Tracks m + A B^T with orthonormal B (rank 3): the basis spans B."""
    g = np.random.default_rng(24)
    n, n_seg, r = 300, 30, 3
    B, _ = np.linalg.qr(g.standard_normal((n_seg, r)))
    A = g.standard_normal((n, r)) * np.array([5.0, 2.0, 0.5])
    m = g.uniform(size=n_seg)
    F = m[None, :] + A @ B.T
    f0, U, sv, lo, hi = (np.asarray(v) for v in build_basis(F, r))
    cosines = np.linalg.svd(U.T @ B, compute_uv=False)
    assert np.all(cosines > 1 - 1e-12)


# ----------------------------------------------------------------------------- statistic


def tiny_score_case(seed: int, with_ties: bool = True):
    """Tiny dyadic problem with exact half-bin ties and out-of-range tracks."""
    g = np.random.default_rng(seed)
    n_seg, n_bins, K, n_tmpl = 4, 64, 3, 8
    t_sft = 64.0                                # bin width 1/64 Hz: dyadic
    P = g.uniform(0.0, 5.0, (n_seg, n_bins))
    f0 = g.integers(10, 50, n_seg) / t_sft
    U = g.integers(-8, 9, (n_seg, K)) / 16.0
    C = (g.integers(-64, 65, (n_tmpl, K)) / 8.0).astype(np.float32)
    if with_ties:
        # template 0 sits on exact half-bins: x = f0 T + 8 U[a, 0] with U[a, 0] = m/16
        U[0, 0] = 1.0 / 16.0
        U[1:, 0] = g.choice([-7, -5, -3, -1, 1, 3, 5, 7], n_seg - 1) / 16.0
        C[0] = 0.0
        C[0, 0] = 0.125
        C[1] = np.float32(1e4)                   # far out of range in every segment
    return P, f0, U, C, t_sft


def check_score_exact(score_tracks):
    from fractions import Fraction
    for seed in range(6):
        P, f0, U, C, t_sft = tiny_score_case(seed)
        got = score_tracks(P, f0, U, C, t_sft, 0, want_bins=True)
        n_seg, n_bins = P.shape
        for j in range(C.shape[0]):
            total = Fraction(0)
            for a in range(n_seg):
                pos = Fraction(float(f0[a]))
                for k in range(U.shape[1]):
                    pos += Fraction(float(C[j, k])) * Fraction(float(U[a, k]))
                pos *= Fraction(t_sft)
                b = round(pos)                      # exact, ties to even
                if 0 <= b < n_bins:
                    assert got["bins"][j, a] == b, (seed, j, a)
                    total += Fraction(float(P[a, b]))
                else:
                    assert got["bins"][j, a] == -1
            assert abs(float(got["stat"][j]) - float(total)) <= 1e-15 * max(1.0, float(total))


def check_score_near_ties_large(score_tracks):
    """Positions near 8000 within 1e-4 of a half-bin: only FP64 positions round right."""
    from fractions import Fraction
    g = np.random.default_rng(33)
    n_seg, n_bins, t_sft = 24, 8193, 163840.0
    P = g.uniform(0.0, 5.0, (n_seg, n_bins))
    base = g.integers(4000, 8000, n_seg) + 0.5 + g.choice([-1, 1], n_seg) * g.uniform(2e-6, 1e-4, n_seg)
    f0 = base / t_sft
    U = g.standard_normal((n_seg, 2)) * 1e-9
    C = g.uniform(-1, 1, (16, 2)).astype(np.float32)
    got = score_tracks(P, f0, U, C, t_sft, 0, want_bins=True)
    for j in range(C.shape[0]):
        for a in range(n_seg):
            pos = Fraction(float(f0[a]))
            for k in range(2):
                pos += Fraction(float(C[j, k])) * Fraction(float(U[a, k]))
            b = round(pos * Fraction(t_sft))
            assert got["bins"][j, a] == (b if 0 <= b < n_bins else -1), (j, a)


def check_score_half_even(score_tracks):
    """Positions exactly at b + 1/2 round to the even neighbour."""
    n_seg, n_bins, t_sft = 6, 32, 8.0
    P = np.arange(n_seg * n_bins, dtype=np.float64).reshape(n_seg, n_bins)
    U = np.ones((n_seg, 1))
    halves = np.array([2.5, 3.5, 4.5, 10.5, 11.5, 0.5])      # bins -> 2, 4, 4, 10, 12, 0
    f0 = halves / t_sft - 0.0
    C = np.zeros((1, 1), dtype=np.float32)
    got = score_tracks(P, f0, U, C, t_sft, 0, want_bins=True)
    assert list(got["bins"][0]) == [2, 4, 4, 10, 12, 0]
    assert got["n_near_tie"] == n_seg
    # a position at -1/2 rounds to -0 (valid bin 0); at n_bins - 1/2 to n_bins (invalid)
    f0b = np.array([-0.5, n_bins - 0.5, -1.5, 1.0, 2.0, 3.0]) / t_sft
    got = score_tracks(P, f0b, U, C, t_sft, 0, want_bins=True)
    assert list(got["bins"][0]) == [0, -1, -1, 1, 2, 3]


def check_score_column_sum(score_tracks):
    g = np.random.default_rng(31)
    n_seg, n_bins, t_sft = 9, 100, 1000.0
    P = g.exponential(size=(n_seg, n_bins))
    for b in (0, 1, 57, 99):
        f0 = np.full(n_seg, b / t_sft)
        got = score_tracks(P, f0, np.zeros((n_seg, 0)), np.zeros((3, 0), np.float32), t_sft, 2)
        assert np.allclose(got["stat"], P[:, b].sum(), rtol=1e-15, atol=0)
        assert list(got["topk_idx"]) == [0, 1]
    # orientation: a track stepping one bin per segment picks the diagonal
    f0 = (np.arange(n_seg) + 10) / t_sft
    got = score_tracks(P, f0, np.zeros((n_seg, 0)), np.zeros((1, 0), np.float32), t_sft, 1)
    assert abs(got["stat"][0] - sum(P[a, a + 10] for a in range(n_seg))) < 1e-12


def check_score_permutation_and_topk(score_tracks):
    g = np.random.default_rng(32)
    n_seg, n_bins, K, n = 12, 300, 3, 500
    t_sft = 1e4
    P = np.round(g.exponential(size=(n_seg, n_bins)), 1)   # coarse values: many exact ties in S
    f0 = g.uniform(0.005, 0.02, n_seg)
    U = g.standard_normal((n_seg, K)) * 2e-3
    C = g.uniform(-1, 1, (n, K)).astype(np.float32)
    C[50:60] = C[7]                                          # duplicated templates tie exactly
    a = score_tracks(P, f0, U, C, t_sft, 40)
    perm = g.permutation(n)
    b = score_tracks(P, f0, U, C[perm], t_sft, 0)
    assert np.array_equal(np.asarray(b["stat"]), np.asarray(a["stat"])[perm])
    order = sorted(range(n), key=lambda j: (-float(a["stat"][j]), j))[:40]
    assert list(a["topk_idx"]) == order
    assert np.array_equal(np.asarray(a["topk_val"]), np.asarray(a["stat"])[order])
    pad = score_tracks(P, f0, U, C[:5], t_sft, 8)
    assert list(pad["topk_idx"][5:]) == [-1, -1, -1]
    assert np.all(np.isneginf(pad["topk_val"][5:]))
    empty = score_tracks(P, f0, U, C[:0], t_sft, 3)
    assert list(empty["topk_idx"]) == [-1, -1, -1] and empty["stat"].size == 0


def check_score_range(score_tracks):
    """k_min/k_max restrict contributing bins; non-finite positions contribute nothing."""
    n_seg, n_bins, t_sft = 3, 50, 10.0
    P = np.ones((n_seg, n_bins))
    f0 = np.array([0.5, 2.0, 4.9])          # bins 5, 20, 49
    U = np.ones((n_seg, 1))
    C = np.array([[0.0], [np.inf], [np.nan], [0.1]], dtype=np.float32)   # last: 6, 21, 50
    got = score_tracks(P, f0, U, C, t_sft, 0, want_bins=True)
    assert list(got["stat"]) == [3.0, 0.0, 0.0, 2.0]
    got = score_tracks(P, f0, U, C, t_sft, 0, k_min=6, k_max=30, want_bins=True)
    assert list(got["stat"]) == [1.0, 0.0, 0.0, 2.0]
    assert list(got["bins"][3]) == [6, 21, -1]


# ------------------------------------------------------------- checker helpers
# Two oracle helpers decide which GPU rows a parity test accepts: the near-tie
# band (either neighbouring bin is correct inside it) and the correctly rounded
# segment sum at given bins (the statistic a GPU row is held to).


def check_near_tie_band(near_tie_mask):
    """Flagged iff |x - floor(x) - 1/2| < 1e-6; never for NaN or +-inf."""
    inside, outside = 0.9e-6, 1.1e-6
    for base in (0.0, 3.0, 117.0, 8000.0, 8192.0, -5.0, -1.0):
        half = base + 0.5
        x = np.array([half, half + inside, half - inside, half + outside, half - outside,
                      base, base + 0.25, base + 0.75])
        got = np.asarray(near_tie_mask(x))
        assert got.dtype == bool
        assert list(got) == [True, True, True, False, False, False, False, False], (base, got)
    x = np.array([np.nan, np.inf, -np.inf, 0.5])
    assert list(np.asarray(near_tie_mask(x))) == [False, False, False, True]


def check_fsum_rows(fsum_rows):
    """Correctly rounded sum over the contributing segments (bin -1: none)."""
    from fractions import Fraction
    g = np.random.default_rng(41)
    n_seg, n_bins = 7, 20
    P = g.uniform(0.0, 1.0, (n_seg, n_bins))
    P[:, -1] = 1e3                       # a -1 bin read as an index would pick these up
    P[0, 3] = 1e16                       # 1e16 + 1 + 1: naive left-to-right sums lose both ones
    P[1, 4] = 1.0
    P[2, 5] = 1.0
    bins = g.integers(0, n_bins - 1, (6, n_seg))
    bins[0, :3] = [3, 4, 5]
    bins[0, 3:] = -1
    bins[1, ::2] = -1
    bins[2] = -1
    got = np.asarray(fsum_rows(P, bins))
    assert got.shape == (bins.shape[0],)
    for j in range(bins.shape[0]):
        want = Fraction(0)
        for a in range(n_seg):
            if bins[j, a] >= 0:
                want += Fraction(float(P[a, bins[j, a]]))
        assert got[j] == float(want), (j, got[j], float(want))
    assert got[0] == 1e16 + 2.0 and got[2] == 0.0
