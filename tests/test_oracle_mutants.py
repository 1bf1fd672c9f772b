"""Plant plausible mistakes in the oracle (CPU only) and check that a pin catches each.

Every mutant patches one step of the oracle module in place (monkeypatch undoes
it afterwards); the pins must then fail.  This shows the pins are sharp enough
that a dropped term, wrong sign, shifted index or transposed operand in the
oracle would not go unnoticed.
"""
import numpy as np
import pytest

import oracle
import oracle.basis as ob
import oracle.score as osc
import oracle.sft as osft
from tests import pins

SFT_PINS = [pins.check_sft_bruteforce, pins.check_sft_parseval, pins.check_sft_sinusoid,
            pins.check_sft_noise_law]
BASIS_PINS = [pins.check_basis_identities, pins.check_basis_full_rank, pins.check_basis_rank_one,
              pins.check_basis_low_rank_recovery]
SCORE_PINS = [pins.check_score_exact, pins.check_score_near_ties_large, pins.check_score_half_even, pins.check_score_column_sum,
              pins.check_score_permutation_and_topk, pins.check_score_range]


def _caught(checks, fn):
    for check in checks:
        try:
            check(fn)
        except (AssertionError, ValueError, IndexError):
            return True
    return False


SFT_MUTANTS = {
    "no_window": ("hann_periodic", lambda n: np.ones(n)),
    "symmetric_hann": ("hann_periodic", lambda n: np.sin(np.pi * np.arange(n) / (n - 1)) ** 2),
    "window_shifted": ("hann_periodic", lambda n: np.sin(np.pi * (np.arange(n) + 0.5) / n) ** 2),
    "norm_missing_2": ("normaliser", lambda w, psd, dt: np.sum(w * w) * psd / dt),
    "norm_sum_w": ("normaliser", lambda w, psd, dt: np.sum(w) * psd / (2.0 * dt)),
    "psd_shifted": ("normaliser", lambda w, psd, dt: np.sum(w * w) * np.roll(psd, 1) / (2.0 * dt)),
    "segments_interleaved": ("segments",
                             lambda x, n: x[: (x.size // n) * n].reshape(n, x.size // n).T),
    "segments_overlap_start": ("segments",
                               lambda x, n: np.stack([x[a * n + 1:(a + 1) * n + 1]
                                                      for a in range(x.size // n - 1)] +
                                                     [x[(x.size // n - 1) * n:(x.size // n) * n]])),
}


@pytest.mark.parametrize("name", sorted(SFT_MUTANTS))
def test_sft_mutant_caught(name, monkeypatch):
    attr, fn = SFT_MUTANTS[name]
    monkeypatch.setattr(osft, attr, fn)
    assert _caught(SFT_PINS, osft.build_sfts), name


def _svd_off_by_one(X, K):
    _, s, vt = np.linalg.svd(X, full_matrices=False)
    return vt[1:K + 1].T.copy(), s[1:]


def _svd_left_padded(X, K):
    u, s, vt = np.linalg.svd(X, full_matrices=False)
    V = vt[:K].T.copy()
    return V[::-1].copy(), s


BASIS_MUTANTS = {
    "uncentred": ("centre_tracks", lambda F: (np.zeros(F.shape[1]), F)),
    "centre_median": ("centre_tracks", lambda F: (np.median(F, axis=0), F - np.median(F, axis=0))),
    "component_off_by_one": ("leading_right_vectors", _svd_off_by_one),
    "segments_reversed": ("leading_right_vectors", _svd_left_padded),
    "no_sign_rule": ("apply_sign_rule", lambda U: -U),
    "box_mean_3std": ("coefficient_box", lambda C: (C.mean(0) - 3 * C.std(0), C.mean(0) + 3 * C.std(0))),
    "box_nearest": ("coefficient_box", lambda C: (np.quantile(C, 0.00135, axis=0, method="nearest"),
                                                  np.quantile(C, 0.99865, axis=0, method="nearest"))),
}


@pytest.mark.parametrize("name", sorted(BASIS_MUTANTS))
def test_basis_mutant_caught(name, monkeypatch):
    attr, fn = BASIS_MUTANTS[name]
    monkeypatch.setattr(ob, attr, fn)
    assert _caught(BASIS_PINS, ob.build_basis), name


_orig_positions = osc.track_positions
_orig_bins = osc.chosen_bins


def _pos_no_f0(f0, U, c, t):
    return _orig_positions(np.zeros_like(np.asarray(f0, dtype=np.float64)), U, c, t)


def _pos_no_T(f0, U, c, t):
    return _orig_positions(f0, U, c, 1.0) * 1.0


def _pos_U_reversed(f0, U, c, t):
    return _orig_positions(f0, np.asarray(U)[::-1], c, t)


def _pos_sign(f0, U, c, t):
    return _orig_positions(f0, -np.asarray(U, dtype=np.float64), c, t)


def _pos_fp32(f0, U, c, t):
    return _orig_positions(f0, U, c, t).astype(np.float32).astype(np.float64)


def _bins_floor(x, n_bins, k_min=0, k_max=None):
    return _orig_bins(np.floor(x), n_bins, k_min, k_max)


def _bins_half_up(x, n_bins, k_min=0, k_max=None):
    return _orig_bins(np.floor(x + 0.5), n_bins, k_min, k_max)


def _bins_clamped(x, n_bins, k_min=0, k_max=None):
    k_max = n_bins - 1 if k_max is None else k_max
    xs = np.where(np.isfinite(x), x, 0.0)
    b = np.clip(np.rint(xs), k_min, k_max).astype(np.int64)
    return b, np.isfinite(x)


def _bins_off_by_one_range(x, n_bins, k_min=0, k_max=None):
    return _orig_bins(x, n_bins + 1, k_min, None if k_max is None else k_max + 1)


def _topk_desc_index(stat, top_k):
    stat = np.asarray(stat, dtype=np.float64)
    n = stat.size
    order = np.lexsort((-np.arange(n), -stat))[: min(top_k, n)]
    vals = np.full(top_k, -np.inf)
    idx = np.full(top_k, -1, dtype=np.int64)
    vals[: order.size] = stat[order]
    idx[: order.size] = order
    return vals, idx


def _topk_ascending(stat, top_k):
    stat = np.asarray(stat, dtype=np.float64)
    n = stat.size
    order = np.lexsort((np.arange(n), stat))[: min(top_k, n)]
    vals = np.full(top_k, -np.inf)
    idx = np.full(top_k, -1, dtype=np.int64)
    vals[: order.size] = stat[order]
    idx[: order.size] = order
    return vals, idx


SCORE_MUTANTS = {
    "dropped_f0": ("track_positions", _pos_no_f0),
    "missing_T": ("track_positions", _pos_no_T),
    "segments_reversed": ("track_positions", _pos_U_reversed),
    "basis_sign": ("track_positions", _pos_sign),
    "fp32_positions": ("track_positions", _pos_fp32),
    "floor": ("chosen_bins", _bins_floor),
    "half_up": ("chosen_bins", _bins_half_up),
    "clamped_edges": ("chosen_bins", _bins_clamped),
    "range_off_by_one": ("chosen_bins", _bins_off_by_one_range),
    "topk_tiebreak": ("topk_order", _topk_desc_index),
    "topk_ascending": ("topk_order", _topk_ascending),
}


@pytest.mark.parametrize("name", sorted(SCORE_MUTANTS))
def test_score_mutant_caught(name, monkeypatch):
    attr, fn = SCORE_MUTANTS[name]
    monkeypatch.setattr(osc, attr, fn)
    assert _caught(SCORE_PINS, osc.score_tracks), name


# The checker helpers: a band wider than 1e-6 would excuse real bin errors; a
# sum that counts non-contributing (-1) bins or rounds naively would hold GPU
# rows to a wrong statistic.
def _fsum_counts_invalid(P, bins):
    P = np.asarray(P, dtype=np.float64)
    return np.array([sum(P[a, b] for a, b in enumerate(row)) for row in bins])


def _fsum_naive(P, bins):
    P = np.asarray(P, dtype=np.float64)
    out = np.zeros(bins.shape[0])
    for j in range(bins.shape[0]):
        acc = 0.0
        for a, b in enumerate(bins[j]):
            if b >= 0:
                acc += P[a, b]
        out[j] = acc
    return out


def _near_tie_closed_band(x):
    finite = np.isfinite(x)
    xs = np.where(finite, x, 0.0)
    return finite & (np.abs(xs - np.floor(xs) - 0.5) <= osc.NEAR_TIE_BAND * 1.2)


def _near_tie_nonfinite(x):
    xs = np.nan_to_num(np.asarray(x, dtype=np.float64), nan=0.5, posinf=0.5, neginf=0.5)
    return np.abs(xs - np.floor(xs) - 0.5) < osc.NEAR_TIE_BAND


@pytest.mark.parametrize("band", [1e-3, 1e-5, 1e-7])
def test_near_tie_band_mutant_caught(band, monkeypatch):
    monkeypatch.setattr(osc, "NEAR_TIE_BAND", band)
    assert _caught([pins.check_near_tie_band], osc.near_tie_mask), band


@pytest.mark.parametrize("fn", [_near_tie_closed_band, _near_tie_nonfinite])
def test_near_tie_mutant_caught(fn):
    assert _caught([pins.check_near_tie_band], fn), fn.__name__


@pytest.mark.parametrize("fn", [_fsum_counts_invalid, _fsum_naive])
def test_fsum_rows_mutant_caught(fn):
    assert _caught([pins.check_fsum_rows], fn), fn.__name__


# ---------------------------------------------------------------- search (Eq. (11))
import oracle.search as osr
from tests import pins_search

SEARCH_PINS = [pins_search.check_de_trial_closed_form, pins_search.check_seed_closed_form,
               pins_search.check_de_acceptance, pins_search.check_seed_keeps_best]


def _search_caught(monkeypatch, attr, fn):
    monkeypatch.setattr(osr, attr, fn)
    targets = {pins_search.check_de_trial_closed_form: lambda: osr.de_trials,
               pins_search.check_seed_closed_form: lambda: osr.seed_candidates,
               pins_search.check_de_acceptance: lambda: osr.de_generation,
               pins_search.check_seed_keeps_best: lambda: osr.seed_population}
    for check, target in targets.items():
        try:
            check(target())
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def _trials_sign(f0, U, coeffs, r1, r2, F):
    return _orig_trials(f0, U, coeffs, r2, r1, F)


def _trials_no_F(f0, U, coeffs, r1, r2, F):
    return _orig_trials(f0, U, coeffs, r1, r2, np.ones_like(np.asarray(F, dtype=np.float64)))


def _project_transpose(f0, U, tracks):
    return (np.asarray(tracks) - np.asarray(f0)[None, :]) @ np.asarray(U)


def _in_prior_strict(coeffs, lo, hi):
    c = np.asarray(coeffs, dtype=np.float32).astype(np.float64)
    return np.all((c > np.asarray(lo)[None, :]) & (c < np.asarray(hi)[None, :]), axis=1)


def _in_prior_always(coeffs, lo, hi):
    return np.ones(np.asarray(coeffs).shape[0], dtype=bool)


def _seed_last_segment(f0, U, draws, f_init):
    f = osr.tracks_of(f0, U, draws)
    moved = f + (np.asarray(f_init) - f[:, -1])[:, None]
    return osr.project(f0, U, moved).astype(np.float32)


def _seed_absolute(f0, U, draws, f_init):
    f = osr.tracks_of(f0, U, draws)
    return osr.project(f0, U, f + np.asarray(f_init)[:, None]).astype(np.float32)


def _tracks_no_f0(f0, U, coeffs):
    return np.asarray(coeffs, dtype=np.float32).astype(np.float64) @ np.asarray(U).T


_orig_trials = osr.de_trials
_orig_generation = osr.de_generation


def _generation_ge(P, f0, U, lo, hi, coeffs, stat, r1, r2, F, t, k_min=0, k_max=None):
    out = _orig_generation(P, f0, U, lo, hi, coeffs, stat, r1, r2, F, t, k_min, k_max)
    acc = out["in_prior"] & (out["trial_stat"] >= np.asarray(stat))
    out["accepted"] = acc
    out["coeffs"] = np.where(acc[:, None], out["trial"], coeffs)
    out["stat"] = np.where(acc, out["trial_stat"], stat)
    return out


def _keep_worst(P, f0, U, draws, f_init, t, n_keep, k_min=0, k_max=None):
    cand = osr.seed_candidates(f0, U, draws, f_init)
    st = osr.score_tracks(P, f0, U, cand, t, 0)["stat"]
    idx = np.lexsort((np.arange(st.size), st))[:n_keep]
    return cand[idx], st[idx], idx


SEARCH_MUTANTS = {
    "trial_sign": ("de_trials", _trials_sign),
    "trial_no_F": ("de_trials", _trials_no_F),
    "project_transpose": ("project", _project_transpose),
    "prior_strict": ("in_prior", _in_prior_strict),
    "prior_ignored": ("in_prior", _in_prior_always),
    "seed_last_segment": ("seed_candidates", _seed_last_segment),
    "seed_absolute": ("seed_candidates", _seed_absolute),
    "tracks_no_f0": ("tracks_of", _tracks_no_f0),
    "accept_ties": ("de_generation", _generation_ge),
    "keep_worst": ("seed_population", _keep_worst),
}


@pytest.mark.parametrize("name", sorted(SEARCH_MUTANTS))
def test_search_mutant_caught(name, monkeypatch):
    attr, fn = SEARCH_MUTANTS[name]
    assert _search_caught(monkeypatch, attr, fn), name


def _shift_first_rows(f0, U, n):
    return np.asarray(f0)[:n], np.asarray(U)[:n]


def _moments_population(best):
    b = np.asarray(best, dtype=np.float64)
    return b.mean(axis=0), b.std(axis=0)


def _best_nan_first(stat):
    s = np.asarray(stat, dtype=np.float64)
    return int(np.lexsort((np.arange(s.size), -np.nan_to_num(s, nan=np.inf)))[0])


def _best_last_tie(stat):
    s = np.asarray(stat, dtype=np.float64)
    key = np.where(np.isnan(s), -np.inf, s)
    return int(np.lexsort((-np.arange(s.size), -key))[0])


@pytest.mark.parametrize("check,fn", [
    (pins_search.check_shifted_basis, _shift_first_rows),
    (pins_search.check_noise_moments, _moments_population),
    (pins_search.check_best_walker, _best_nan_first),
    (pins_search.check_best_walker, _best_last_tie),
])
def test_progressive_mutant_caught(check, fn):
    assert _caught([check], fn), fn.__name__


# ---------------------------------------------------------------- harmonics (Sec. IV)
import oracle.harmonics as ohm
from tests import pins_harmonics

HARMONIC_PINS = [pins_harmonics.check_harmonics_exact, pins_harmonics.check_harmonics_constant_track,
                 pins_harmonics.check_harmonics_additive]


def _hpos_round_first(x, ratios):
    r = np.asarray(ratios, dtype=np.float64)
    return r[:, None, None] * np.rint(np.asarray(x, dtype=np.float64))[None, :, :]


def _hpos_inverse(x, ratios):
    r = np.asarray(ratios, dtype=np.float64)
    return np.asarray(x, dtype=np.float64)[None, :, :] / r[:, None, None]


def _hpos_drop_first(x, ratios):
    r = np.asarray(ratios, dtype=np.float64)[1:]
    return r[:, None, None] * np.asarray(x, dtype=np.float64)[None, :, :]


@pytest.mark.parametrize("fn", [_hpos_round_first, _hpos_inverse, _hpos_drop_first])
def test_harmonic_mutant_caught(fn, monkeypatch):
    monkeypatch.setattr(ohm, "harmonic_positions", fn)
    assert _caught(HARMONIC_PINS, ohm.score_harmonics), fn.__name__


# ---------------------------------------------------------------- linear chirp (Sec. II B)
import oracle.chirp as och
from tests import pins_chirp

_orig_template = och.chirp_template_bins
_orig_segment = och.segment_statistic


def _chirp_checks():
    return [lambda: pins_chirp.check_template_bruteforce(och.chirp_template_bins),
            lambda: pins_chirp.check_template_no_derivative(och.chirp_template_bins),
            lambda: pins_chirp.check_one_bin_is_nearest_bin_power(och.score_chirp, och.build_sfts_complex,
                                                                  och.inverse_sqrt_psd),
            lambda: pins_chirp.check_matched_chirp(och.segment_statistic, och.build_sfts_complex,
                                                   och.inverse_sqrt_psd, och.chirp_template_bins),
            lambda: pins_chirp.check_track_derivatives(och.track_derivatives),
            lambda: pins_chirp.check_validity_and_cutoffs(och.score_chirp, och.build_sfts_complex,
                                                          och.inverse_sqrt_psd)]


def _template_beta_sign(d0, beta, p):
    return _orig_template(d0, -beta, p)


def _template_rect(d0, beta, p):
    m = np.arange(-p, p + 1)
    u, wt = och._gauss_grid(abs(d0) + p + abs(beta) + 1.0)
    g = wt * np.exp(1j * (2.0 * np.pi * d0 * u + np.pi * beta * u * u))
    return np.exp(-2j * np.pi * np.outer(m, u)) @ g


def _segment_no_sign(Z_row, isq, f, fdot, t_sft, p_half):
    # the (-1)^k of the segment-start time origin dropped
    orig = och.chirp_template_bins
    k0 = int(np.rint(f * t_sft))
    def tpl(d0, beta, p):
        m = np.arange(-p, p + 1)
        return orig(d0, beta, p) * np.where((k0 + m) % 2 == 0, 1.0, -1.0)
    och.chirp_template_bins = tpl
    try:
        return _orig_segment(Z_row, isq, f, fdot, t_sft, p_half)
    finally:
        och.chirp_template_bins = orig


def _segment_no_weight(Z_row, isq, f, fdot, t_sft, p_half):
    return _orig_segment(Z_row, np.where(isq > 0, 1.0, 0.0), f, fdot, t_sft, p_half)


def _derivative_forward(f, t_sft):
    f = np.asarray(f, dtype=np.float64)
    fd = np.empty_like(f)
    fd[..., :-1] = (f[..., 1:] - f[..., :-1]) / t_sft
    fd[..., -1] = fd[..., -2]
    fdd = np.zeros_like(f)
    return fd, fdd


def _valid_T2(f, fdot, fddot, t_sft, f_min=och.F_MIN, fdot_min=och.FDOT_MIN):
    return (np.abs(fddot) * t_sft ** 2 / 6.0 <= 1.0) & (f >= f_min) & (fdot >= fdot_min)


def _valid_abs_fdot(f, fdot, fddot, t_sft, f_min=och.F_MIN, fdot_min=och.FDOT_MIN):
    return (np.abs(fddot) * t_sft ** 3 / 6.0 <= 1.0) & (f >= f_min) & (np.abs(fdot) >= fdot_min)


@pytest.mark.parametrize("attr,fn", [
    ("chirp_template_bins", _template_beta_sign), ("chirp_template_bins", _template_rect),
    ("segment_statistic", _segment_no_sign), ("segment_statistic", _segment_no_weight),
    ("track_derivatives", _derivative_forward), ("segment_valid", _valid_T2), ("segment_valid", _valid_abs_fdot),
])
def test_chirp_mutant_caught(attr, fn, monkeypatch):
    monkeypatch.setattr(och, attr, fn)
    caught = False
    for check in _chirp_checks():
        try:
            check()
        except (AssertionError, ValueError, IndexError):
            caught = True
            break
    assert caught, fn.__name__
