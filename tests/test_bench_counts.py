"""Host bookkeeping of bench.py against the oracle (CPU).

The chirp form's roofline counts the template-segment pairs the statistic
evaluates; that count must be the oracle's: valid segments (fddot limit and
cut-offs of Sec. II D) whose central bin lies in the row.
"""
import importlib.util
import os

import numpy as np

import oracle
import oracle.chirp as och

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_chirp_evaluated_segments_matches_oracle():
    bench = _bench()
    g = np.random.default_rng(11)
    n_seg, K, T, n_bins = 23, 4, 1000.0, 900
    f0 = np.linspace(0.2, 0.7, n_seg)
    U = g.standard_normal((n_seg, K)) * 0.05
    C = g.uniform(-3, 3, (5000, K)).astype(np.float32)
    C[:50] *= 30.0                                    # cuts, out-of-row central bins
    for f_min, fdot_min in ((och.F_MIN, och.FDOT_MIN), (0.3, 0.0), (-np.inf, -np.inf)):
        f = oracle.track_positions(f0, U, C, 1.0)
        fd, fdd = och.track_derivatives(f, T)
        k0 = np.rint(f * T)
        want = och.segment_valid(f, fd, fdd, T, f_min, fdot_min) & (k0 >= 0) & (k0 < n_bins)
        got = bench.chirp_evaluated_segments(f0, U, C, T, n_bins, f_min, fdot_min, chunk=777)
        assert got == int(want.sum())
        assert 0 < got < C.size
