"""Search driver: the population search of Sec. II D on the library's kernels.

The paper searches for the coefficients (and the plunge time) that maximise
the statistic: for each of 48 observed durations, growing from 0.1 yr, the
one-year basis is shifted by a whole number of segments so that the track
ends at the end of the data (plunge at the end of the observation), a
population is seeded (1024 candidates, the best 512 kept) and improved by
525 iterations of differential evolution in track space (Eq. (11)); every
duration's best statistic is normalised by the mean and standard deviation
of the same search on noise-only data, and the best normalised value over
durations is the detection statistic.

Here every duration is one chain and all chains advance together: a pair of
generations is two launches over every chain (``SearchPlan.generations``:
each forms, projects and scores every walker's trial and selects, reading
one copy of the population and writing the other), and a run of generations
is captured into one HIP graph and replayed.  This module only
builds the chain views (pointer offsets into one spectrogram and one basis)
and launches; the arithmetic is in the library's kernels.  Random numbers
(seed candidates, initial frequencies, partners, weights) are inputs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import Chain, SearchPlan, Spectrogram, search_seed, search_noise_moments


def progressive_durations(n_seg: int, n_chunks: int = 48, start_frac: float = 0.1) -> list[int]:
    """Segment counts of the observed durations: from start_frac of the data
    to all of it in n_chunks near-equal steps (the paper's 0.1 yr growing by
    about a week, 48 durations)."""
    first = max(1, int(round(start_frac * n_seg)))
    if n_chunks == 1:
        return [n_seg]
    out = [int(round(first + (n_seg - first) * c / (n_chunks - 1))) for c in range(n_chunks)]
    return sorted(set(out))


def shifted_chain(spec: Spectrogram, f0, U, box_lo, box_hi, n: int, n_walkers: int, k_min: int = 0) -> Chain:
    """A chain on the first n segments of spec whose basis is the full basis
    shifted by n_seg - n segments (its last rows), so every track ends where
    the data end."""
    import torch
    N = spec.n_seg
    if not 1 <= n <= N:
        raise ValueError("duration outside the spectrogram")
    K = int(U.shape[1])
    dev = spec.data.device
    sub = Spectrogram(spec.data[:n], spec.n_bins, spec.t_sft)
    # the shifted rows are copied: a view of f0 starting at an odd row would
    # break the library's 16-byte alignment rule
    return Chain(sub, f0[N - n:].clone(), U[N - n:].clone(), box_lo, box_hi,
                 torch.zeros((n_walkers, K), dtype=torch.float32, device=dev),
                 torch.zeros(n_walkers, dtype=torch.float32, device=dev), k_min=k_min)


@dataclass
class SearchRun:
    chains: list
    plan: SearchPlan
    graph: object
    gens_per_replay: int


def prepare(chains: list, K: int, draws, f_init, r1, r2, F, precision: str = "plain") -> SearchRun:
    """Seed every chain and capture the generations of r1, r2, F (shape
    (n_gen, total walkers)) into one HIP graph (replay() runs them all)."""
    import torch
    search_seed(chains, K, draws, f_init, precision=precision)
    plan = SearchPlan(chains, K, precision=precision)
    # warm the kernels outside capture, on a side stream
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    saved = [(c.coeffs.clone(), c.stat.clone()) for c in chains]
    with torch.cuda.stream(side):
        plan.generation(r1[0], r2[0], F[0], stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for c, (C, S) in zip(chains, saved):
        c.coeffs.copy_(C)
        c.stat.copy_(S)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.generations(r1, r2, F)
    return SearchRun(list(chains), plan, graph, int(r1.shape[0]))


def noise_moments(best_stats) -> tuple:
    """Mean and standard deviation over noise-only realisations of every
    chain's best statistic: best_stats is a (n_real, n_chains) float32 device
    tensor; returns two float64 device tensors (n_chains,)."""
    return search_noise_moments(best_stats)
