"""Numbers the paper prints that the segmentation must reproduce (CPU only)."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_segment_counts_from_paper():
    g = json.load(open(os.path.join(HERE, "golden", "paper_segment_counts.json")))
    n = int(round(g["year_s"] / g["dt"]))
    x = np.zeros(n)
    for case in g["cases"]:
        n_sft = int(round(case["t_sft"] / g["dt"]))
        P = oracle.build_sfts(x, g["dt"], n_sft, np.ones(n_sft // 2 + 1))
        assert P.shape[0] == case["n_seg"], case
        # the bin width is 1/T_SFT
        f = oracle.sft_bin_frequencies(n_sft, g["dt"])
        assert abs(f[1] - 1.0 / case["t_sft"]) < 1e-18
    # 12 SFTs of 5e4 s are about a week; 0.1 yr is 63 whole SFTs
    assert abs(g["chunk_step_sfts"] * 5e4 / 86400 - g["chunk_step_days_approx"]) < 0.1
    assert int(g["first_chunk_years"] * g["year_s"] // 5e4) == 63
