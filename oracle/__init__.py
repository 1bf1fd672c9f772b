"""Plain FP64 CPU oracle for the semi-coherent single-harmonic track search.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link this package: only the test suite, the smoke check of the entry-point
module and the CPU-baseline leg of the benchmark use it.  It shares no code with
the HIP library and imports nothing from it.

Each function is the plain definition of one step, written from the paper:

* ``build_sfts``   -- SFT power of each segment, normalised by the known PSD
                      (Sec. II B, the SFT decomposition behind Eq. (3); Eq. (7);
                      Sec. II F for the data);
* ``build_basis``  -- centred SVD basis of training tracks and the
                      coefficient box (Sec. II C, Eqs. (9)-(10));
* ``score_tracks`` -- the semi-coherent statistic Eq. (6) in its nearest-bin
                      limit, summed over segments, plus the top-k selection of
                      Sec. II D;
* ``search``       -- the population search of Sec. II D: seeding and the
                      track-space differential-evolution step of Eq. (11),
                      the shifted basis and noise normalisation of the
                      progressive-duration search;
* ``harmonics``    -- the multi-harmonic statistic proposed in Sec. IV;
* ``chirp``        -- the linear-chirp statistic of Sec. II B over 2P + 1 bins
                      (Eqs. (4)-(7)) with the validity cut and cut-offs.

Every function is pinned by the CPU tests against closed forms, brute force on
tiny inputs and distributional laws (see the test modules); none is marked
"parity unpinned".
"""
from .sft import build_sfts, hann_periodic, sft_bin_frequencies
from .basis import build_basis, BOX_Q_LO, BOX_Q_HI
from .score import (score_tracks, track_positions, chosen_bins, near_tie_mask,
                    topk_order, score_tracks_exact, NEAR_TIE_BAND)
from . import search, harmonics, chirp

__all__ = [
    "build_sfts", "hann_periodic", "sft_bin_frequencies",
    "build_basis", "BOX_Q_LO", "BOX_Q_HI",
    "score_tracks", "track_positions", "chosen_bins", "near_tie_mask", "topk_order",
    "score_tracks_exact", "NEAR_TIE_BAND", "search", "harmonics", "chirp",
]
