"""The oracle against its pins (CPU only)."""
import numpy as np
import pytest

import oracle
from tests import pins


def test_sft_bruteforce_dft():
    pins.check_sft_bruteforce(oracle.build_sfts)


def test_sft_parseval():
    pins.check_sft_parseval(oracle.build_sfts)


def test_sft_sinusoid_closed_form():
    pins.check_sft_sinusoid(oracle.build_sfts)


def test_sft_noise_exp1_and_gamma():
    pins.check_sft_noise_law(oracle.build_sfts)


def test_noise_gamma_through_statistic():
    pins.check_sft_noise_law(oracle.build_sfts, oracle.score_tracks)


def test_basis_identities():
    pins.check_basis_identities(oracle.build_basis)


def test_basis_full_rank():
    pins.check_basis_full_rank(oracle.build_basis)


def test_basis_rank_one_closed_form():
    pins.check_basis_rank_one(oracle.build_basis)


def test_basis_low_rank_recovery():
    pins.check_basis_low_rank_recovery(oracle.build_basis)


def test_score_exact_bruteforce():
    pins.check_score_exact(oracle.score_tracks)


def test_score_exact_matches_fraction_oracle():
    for seed in range(3):
        P, f0, U, C, t = pins.tiny_score_case(seed)
        s_exact, b_exact = oracle.score_tracks_exact(P, f0, U, C, t)
        got = oracle.score_tracks(P, f0, U, C, t, 0, want_bins=True)
        assert np.array_equal(got["bins"], b_exact)
        assert np.allclose(got["stat"], s_exact, rtol=1e-15, atol=0)


def test_score_near_ties_large():
    pins.check_score_near_ties_large(oracle.score_tracks)


def test_score_half_even():
    pins.check_score_half_even(oracle.score_tracks)


def test_score_column_sum():
    pins.check_score_column_sum(oracle.score_tracks)


def test_score_permutation_and_topk():
    pins.check_score_permutation_and_topk(oracle.score_tracks)


def test_score_range_and_nonfinite():
    pins.check_score_range(oracle.score_tracks)


def test_near_tie_band():
    pins.check_near_tie_band(oracle.near_tie_mask)


def test_fsum_rows():
    from oracle.score import fsum_rows
    pins.check_fsum_rows(fsum_rows)


def test_search_de_trial_closed_form():
    import oracle.search as osr
    from tests import pins_search
    pins_search.check_de_trial_closed_form(osr.de_trials)


def test_search_seed_closed_form():
    import oracle.search as osr
    from tests import pins_search
    pins_search.check_seed_closed_form(osr.seed_candidates)


def test_search_de_acceptance():
    import oracle.search as osr
    from tests import pins_search
    pins_search.check_de_acceptance(osr.de_generation)


def test_search_seed_keeps_best():
    import oracle.search as osr
    from tests import pins_search
    pins_search.check_seed_keeps_best(osr.seed_population)


def test_search_progressive_pieces():
    import oracle.search as osr
    from tests import pins_search
    pins_search.check_shifted_basis(osr.shifted_basis)
    pins_search.check_noise_moments(osr.noise_moments)
    pins_search.check_best_walker(osr.best_walker)


def test_harmonics_pins():
    import oracle.harmonics as ohm
    from tests import pins_harmonics
    pins_harmonics.check_harmonics_exact(ohm.score_harmonics)
    pins_harmonics.check_harmonics_constant_track(ohm.score_harmonics)
    pins_harmonics.check_harmonics_additive(ohm.score_harmonics)


def test_chirp_template_against_bruteforce_dft():
    import oracle.chirp as oc
    from tests import pins_chirp
    pins_chirp.check_template_bruteforce(oc.chirp_template_bins)
    pins_chirp.check_template_no_derivative(oc.chirp_template_bins)


def test_chirp_statistic_pins():
    import oracle.chirp as oc
    from tests import pins_chirp
    pins_chirp.check_one_bin_is_nearest_bin_power(oc.score_chirp, oc.build_sfts_complex, oc.inverse_sqrt_psd)
    pins_chirp.check_matched_chirp(oc.segment_statistic, oc.build_sfts_complex, oc.inverse_sqrt_psd,
                                   oc.chirp_template_bins)
    pins_chirp.check_track_derivatives(oc.track_derivatives)
    pins_chirp.check_validity_and_cutoffs(oc.score_chirp, oc.build_sfts_complex, oc.inverse_sqrt_psd)


def test_chirp_complex_sft_power_is_build_sfts():
    import oracle.chirp as oc
    g = np.random.default_rng(3)
    x = g.standard_normal(5 * 600)
    psd = g.uniform(1, 3, 301)
    psd[7] = 0.0
    Z = oc.build_sfts_complex(x, 2.0, 600, psd)
    assert np.allclose(np.abs(Z) ** 2, oracle.build_sfts(x, 2.0, 600, psd), rtol=1e-12, atol=0)


def test_oracle_is_isolated():
    """The oracle imports nothing from the HIP library package."""
    import ast, pathlib
    root = pathlib.Path(oracle.__file__).parent
    for path in root.glob("*.py"):
        tree = ast.parse(path.read_text())
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom) and node.module:
                names = [node.module]
            for n in names:
                assert not n.startswith("paper_2510_20891_amd"), path
                assert not n.startswith("synth"), path
