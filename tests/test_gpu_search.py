"""Population search (Sec. II D, Eq. (11)) on the GPU against the FP64 oracle.

Three chains search the one-year stream at three observed durations (192,
140 and 63 segments, the one-year basis shifted so that each track ends at
the end of its data), 1024 seed candidates and 512 walkers each, K = 8.

* Seeding: every walker the GPU keeps is one of the oracle's moved-and-
  projected candidates, bit for bit (at most a handful may differ in the last
  bit of a coefficient, through the pseudo-inverse of an ill-conditioned
  shifted basis; their positions must then agree within 1e-6 bin), the kept
  set is the oracle's best 512 (up to entries within 2e-5 of the 512th), and
  statistics agree within 1e-5 except at near-tie positions.
* Generations: from a state both sides share (the oracle's), one generation
  with shared draws; acceptance agrees wherever it is decided by more than
  2e-5 relative and by no near-tie position; accepted walkers hold the
  oracle's trial, rejected walkers are unchanged.
* A HIP graph of several generations replays to the eager result, every
  replay; invalid partner indices leave a walker unchanged; the best walker
  per chain and its normalised statistic match a sort.
"""
import numpy as np
import pytest

import oracle
import oracle.search as osr
import synth

pytestmark = pytest.mark.gpu

DURATIONS = (192, 140, 63)
K, N_DRAW, N_WALK = 8, 1024, 512


def _t(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def world(gpu_lib):
    import torch
    emri = gpu_lib
    st = synth.stream_config1(stream=0)
    f0, U, sv, lo, hi = oracle.build_basis(st["tracks"], K)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]))
    torch.cuda.synchronize()
    P = _np(spec.power()).astype(np.float64)
    N = spec.n_seg
    chains, host = [], []
    for n in DURATIONS:
        sub = emri.Spectrogram(spec.data[:n], spec.n_bins, spec.t_sft)
        chains.append(emri.Chain(sub, _t(f0[N - n:]), _t(U[N - n:]), _t(lo), _t(hi),
                                 torch.zeros((N_WALK, K), dtype=torch.float32, device="cuda"),
                                 torch.zeros(N_WALK, dtype=torch.float32, device="cuda")))
        host.append(dict(P=P[:n], f0=f0[N - n:], U=U[N - n:]))
    draws, finit = zip(*[synth.search_seed_draws(5, c, N_DRAW, lo, hi) for c in range(len(DURATIONS))])
    return dict(emri=emri, chains=chains, host=host, lo=lo, hi=hi, t=spec.t_sft,
                draws=np.concatenate(draws), finit=np.concatenate(finit), spec=spec)


def _positions(h, C, t):
    return oracle.track_positions(h["f0"], h["U"], C, t)


def test_seed_matches_oracle(world):
    import torch
    emri, chains, t = world["emri"], world["chains"], world["t"]
    emri.search_seed(chains, K, _t(world["draws"]), _t(world["finit"]))
    torch.cuda.synchronize()
    for c, (ch, h) in enumerate(zip(chains, world["host"])):
        d = world["draws"][c * N_DRAW:(c + 1) * N_DRAW]
        fi = world["finit"][c * N_DRAW:(c + 1) * N_DRAW]
        cand = osr.seed_candidates(h["f0"], h["U"], d, fi)
        full = oracle.score_tracks(h["P"], h["f0"], h["U"], cand, t, 0)["stat"]
        gpu_c, gpu_s = _np(ch.coeffs), _np(ch.stat)
        # map every kept walker to its candidate
        key = {cand[j].tobytes(): j for j in range(N_DRAW)}
        idx = np.array([key.get(r.tobytes(), -1) for r in gpu_c])
        loose = np.flatnonzero(idx < 0)
        assert loose.size <= 5, loose.size
        xc = _positions(h, cand, t)
        for i in loose:                              # last-bit differences of the projection
            dx = np.abs(_positions(h, gpu_c[i:i + 1], t)[0][None, :] - xc).max(axis=1)
            j = int(np.argmin(dx))
            assert dx[j] <= 1e-6, dx[j]
            idx[i] = j
        assert len(set(idx.tolist())) == N_WALK
        near = oracle.near_tie_mask(xc).any(axis=1)
        ok = ~near[idx]
        rel = np.abs(gpu_s - full[idx]) / np.abs(full[idx])
        assert rel[ok].max() <= 1e-5, rel[ok].max()
        # the kept set is the oracle's best N_WALK, in (-S, index) order
        vals, order = oracle.topk_order(full, N_WALK)
        kth = vals[-1]
        band = 2e-5 * abs(kth)
        sure = set(order[vals > kth + band].tolist())
        assert sure <= set(idx.tolist())
        assert not np.any((full[idx] < kth - band) & ~near[idx])
        assert np.all(np.diff(gpu_s) <= 0)


def _gen_draws(c, gen):
    return synth.search_generation_draws(5, c, gen, N_WALK)


def _set_state(chains, states):
    for ch, (C, S) in zip(chains, states):
        ch.coeffs.copy_(_t(C))
        ch.stat.copy_(_t(S.astype(np.float32)))


def test_generations_match_oracle(world):
    import torch
    emri, chains, t, lo, hi = world["emri"], world["chains"], world["t"], world["lo"], world["hi"]
    # shared starting state: the oracle's seed populations
    states = []
    for c, h in enumerate(world["host"]):
        d = world["draws"][c * N_DRAW:(c + 1) * N_DRAW]
        fi = world["finit"][c * N_DRAW:(c + 1) * N_DRAW]
        C, S, _ = osr.seed_population(h["P"], h["f0"], h["U"], d, fi, t, N_WALK)
        states.append((C, S))
    plan = emri.SearchPlan(chains, K)
    n_acc = 0
    for gen in range(4):
        _set_state(chains, states)
        draws = [_gen_draws(c, gen) for c in range(len(chains))]
        r1 = _t(np.concatenate([d[0] for d in draws]))
        r2 = _t(np.concatenate([d[1] for d in draws]))
        F = _t(np.concatenate([d[2] for d in draws]))
        acc = torch.full((len(chains) * N_WALK,), -1, dtype=torch.int32, device="cuda")
        plan.generation(r1, r2, F, acc)
        torch.cuda.synchronize()
        acc = _np(acc).reshape(len(chains), N_WALK)
        new_states = []
        for c, (ch, h) in enumerate(zip(chains, world["host"])):
            C0, S0 = states[c]
            S0f = S0.astype(np.float32).astype(np.float64)          # the GPU walkers hold FP32 statistics
            o = osr.de_generation(h["P"], h["f0"], h["U"], lo, hi, C0, S0f, *draws[c], t)
            near = (oracle.near_tie_mask(_positions(h, o["trial"], t)).any(axis=1)
                    | oracle.near_tie_mask(_positions(h, C0, t)).any(axis=1))
            close = np.abs(o["trial_stat"] - S0f) <= 2e-5 * np.abs(S0f)
            amb = near | (close & o["in_prior"])
            got_c, got_s = _np(ch.coeffs), _np(ch.stat)
            assert np.all((acc[c] == 0) | (acc[c] == 1))
            assert np.array_equal(acc[c][~amb].astype(bool), o["accepted"][~amb]), (gen, c)
            keep = acc[c] == 0
            assert np.array_equal(got_c[keep], C0[keep]) and np.array_equal(got_s[keep], S0.astype(np.float32)[keep])
            took = (acc[c] == 1) & ~amb
            dx = np.abs(_positions(h, got_c[took], t) - _positions(h, o["trial"][took], t))
            assert dx.size == 0 or dx.max() <= 1e-6, dx.max()
            rel = np.abs(got_s[took] - o["trial_stat"][took]) / np.abs(o["trial_stat"][took])
            assert rel.size == 0 or rel.max() <= 1e-5
            n_acc += int(acc[c].sum())
            new_states.append((o["coeffs"], o["stat"]))
        states = new_states
    assert n_acc > 0


def test_fp16_power_generations(world):
    """FP16 spectrogram rows: one generation against the oracle on the same
    FP16 power (acceptance, trials and statistics as above), and fused pairs
    equal to single generations bit for bit."""
    import torch
    emri, t, lo, hi = world["emri"], world["t"], world["lo"], world["hi"]
    st = synth.stream_config1(stream=0)
    f0, U, sv, lo_, hi_ = oracle.build_basis(st["tracks"], K)
    spec = emri.build_sfts(_t(st["x"]), st["dt"], st["n_sft"], _t(st["psd"]), dtype="f16")
    torch.cuda.synchronize()
    P16 = _np(spec.power()).astype(np.float64)
    N = spec.n_seg
    chains, host, states = [], [], []
    for c, n in enumerate((192, 63)):
        sub = emri.Spectrogram(spec.data[:n], spec.n_bins, spec.t_sft)
        chains.append(emri.Chain(sub, _t(f0[N - n:]), _t(U[N - n:]), _t(lo), _t(hi),
                                 torch.zeros((N_WALK, K), dtype=torch.float32, device="cuda"),
                                 torch.zeros(N_WALK, dtype=torch.float32, device="cuda")))
        h = dict(P=P16[:n], f0=f0[N - n:], U=U[N - n:])
        host.append(h)
        d = world["draws"][c * N_DRAW:(c + 1) * N_DRAW]
        fi = world["finit"][c * N_DRAW:(c + 1) * N_DRAW]
        C, S, _ = osr.seed_population(h["P"], h["f0"], h["U"], d, fi, t, N_WALK)
        states.append((C, S))
    plan = emri.SearchPlan(chains, K)
    draws = [_gen_draws(c, 40) for c in range(len(chains))]
    r1, r2, F = (_t(np.concatenate([d[i] for d in draws])) for i in range(3))
    _set_state(chains, states)
    acc = torch.full((len(chains) * N_WALK,), -1, dtype=torch.int32, device="cuda")
    plan.generation(r1, r2, F, acc)
    torch.cuda.synchronize()
    acc = _np(acc).reshape(len(chains), N_WALK)
    n_acc = 0
    for c, (ch, h) in enumerate(zip(chains, host)):
        C0, S0 = states[c]
        S0f = S0.astype(np.float32).astype(np.float64)
        o = osr.de_generation(h["P"], h["f0"], h["U"], lo, hi, C0, S0f, *draws[c], t)
        near = (oracle.near_tie_mask(_positions(h, o["trial"], t)).any(axis=1)
                | oracle.near_tie_mask(_positions(h, C0, t)).any(axis=1))
        close = np.abs(o["trial_stat"] - S0f) <= 2e-5 * np.abs(S0f)
        amb = near | (close & o["in_prior"])
        assert np.array_equal(acc[c][~amb].astype(bool), o["accepted"][~amb]), c
        took = (acc[c] == 1) & ~amb
        rel = np.abs(_np(ch.stat)[took] - o["trial_stat"][took]) / np.abs(o["trial_stat"][took])
        assert rel.size == 0 or rel.max() <= 1e-5
        n_acc += int(acc[c].sum())
    assert n_acc > 0
    # fused pair == two single generations, bit for bit
    more = [[_gen_draws(c, 41 + g) for c in range(len(chains))] for g in range(2)]
    per_gen = [tuple(_t(np.concatenate([d[i] for d in dg])) for i in range(3)) for dg in more]
    _set_state(chains, states)
    for g in range(2):
        plan.generation(*per_gen[g])
    torch.cuda.synchronize()
    single = [(ch.coeffs.clone(), ch.stat.clone()) for ch in chains]
    _set_state(chains, states)
    plan.generations(*(torch.stack([pg[i] for pg in per_gen]).contiguous() for i in range(3)))
    torch.cuda.synchronize()
    for ch, (C, S) in zip(chains, single):
        assert torch.equal(ch.coeffs, C) and torch.equal(ch.stat, S)


def test_graph_of_generations_replays_to_eager(world):
    import torch
    emri, chains = world["emri"], world["chains"]
    emri.search_seed(chains, K, _t(world["draws"]), _t(world["finit"]))
    torch.cuda.synchronize()
    start = [(ch.coeffs.clone(), ch.stat.clone()) for ch in chains]
    G = 6
    draws = []
    for gen in range(G):
        d = [_gen_draws(c, 100 + gen) for c in range(len(chains))]
        draws.append(tuple(_t(np.concatenate([x[i] for x in d])) for i in range(3)))
    plan = emri.SearchPlan(chains, K)

    def reset():
        for ch, (C, S) in zip(chains, start):
            ch.coeffs.copy_(C)
            ch.stat.copy_(S)

    for gen in range(G):
        plan.generation(*draws[gen])
    torch.cuda.synchronize()
    eager = [(ch.coeffs.clone(), ch.stat.clone()) for ch in chains]
    assert any(not torch.equal(a[0], b[0]) for a, b in zip(eager, start))
    reset()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for gen in range(G):
            plan.generation(*draws[gen], stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        for gen in range(G):
            plan.generation(*draws[gen])
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for ch, (C, S) in zip(chains, eager):
            assert torch.equal(ch.coeffs, C) and torch.equal(ch.stat, S), rep
        # eager work between replays
        plan.best()
        torch.cuda.synchronize()


@pytest.mark.parametrize("G", [1, 2, 5, 6])
def test_fused_generations_equal_single_generations(world, G):
    """search_generations (pairs of generations in one launch each, through a
    second copy of the population) gives the walkers and statistics of G
    search_generation calls bit for bit, eagerly and replayed from a graph;
    an odd G ends with one generation run the single way."""
    import torch
    emri, chains = world["emri"], world["chains"]
    emri.search_seed(chains, K, _t(world["draws"]), _t(world["finit"]))
    torch.cuda.synchronize()
    start = [(ch.coeffs.clone(), ch.stat.clone()) for ch in chains]
    draws = []
    for gen in range(G):
        d = [_gen_draws(c, 300 + gen) for c in range(len(chains))]
        draws.append(tuple(_t(np.concatenate([x[i] for x in d])) for i in range(3)))
    stacked = tuple(torch.stack([dr[i] for dr in draws]).contiguous() for i in range(3))
    plan = emri.SearchPlan(chains, K)

    def reset():
        for ch, (C, S) in zip(chains, start):
            ch.coeffs.copy_(C)
            ch.stat.copy_(S)
        torch.cuda.synchronize()

    for gen in range(G):
        plan.generation(*draws[gen])
    torch.cuda.synchronize()
    single = [(ch.coeffs.clone(), ch.stat.clone()) for ch in chains]
    assert any(not torch.equal(a[0], b[0]) for a, b in zip(single, start))
    reset()
    plan.generations(*stacked)
    torch.cuda.synchronize()
    for ch, (C, S) in zip(chains, single):
        assert torch.equal(ch.coeffs, C) and torch.equal(ch.stat, S)
    graph = torch.cuda.CUDAGraph()
    reset()
    with torch.cuda.graph(graph):
        plan.generations(*stacked)
    for rep in range(2):
        reset()
        graph.replay()
        torch.cuda.synchronize()
        for ch, (C, S) in zip(chains, single):
            assert torch.equal(ch.coeffs, C) and torch.equal(ch.stat, S), rep
        plan.best()
        torch.cuda.synchronize()


def test_invalid_partners_keep_the_walker(world):
    import torch
    emri, chains = world["emri"], world["chains"]
    emri.search_seed(chains, K, _t(world["draws"]), _t(world["finit"]))
    torch.cuda.synchronize()
    before = [(ch.coeffs.clone(), ch.stat.clone()) for ch in chains]
    n = len(chains) * N_WALK
    own = np.tile(np.arange(N_WALK), len(chains)).astype(np.int32)
    r1 = own.copy()                                      # a walker paired with itself
    r2 = ((own + 1) % N_WALK).astype(np.int32)
    r1[::7] = N_WALK + 3                                  # out of range
    r2[::5] = -1
    plan = emri.SearchPlan(chains, K)
    acc = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    plan.generation(_t(r1), _t(r2), _t(np.full(n, 1.0)), acc)
    torch.cuda.synchronize()
    assert int(acc.sum()) == 0
    for ch, (C, S) in zip(chains, before):
        assert torch.equal(ch.coeffs, C) and torch.equal(ch.stat, S)


def test_best_walker_and_normalisation(world):
    import torch
    emri, chains = world["emri"], world["chains"]
    emri.search_seed(chains, K, _t(world["draws"]), _t(world["finit"]))
    chains[1].stat[7] = float("nan")
    chains[2].stat[3] = chains[2].stat[0]                 # a tie: the lower index wins
    torch.cuda.synchronize()
    plan = emri.SearchPlan(chains, K)
    mu = np.array([190.0, 141.0, 64.0])
    sd = np.array([3.0, 2.5, 1.5])
    best = plan.best(_t(mu), _t(sd))
    torch.cuda.synchronize()
    for c, ch in enumerate(chains):
        s = _np(ch.stat).astype(np.float64)
        j = osr.best_walker(s)
        assert int(best["idx"][c]) == j
        assert float(best["stat"][c]) == np.float32(s[j])
        want = osr.normalised(s[j], mu[c], sd[c])
        assert abs(float(best["norm"][c]) - want) <= 1e-12 * abs(mu[c])


def test_noise_moments_match_oracle(world):
    import torch
    emri = world["emri"]
    g = np.random.default_rng(8)
    best = g.normal(150.0, 4.0, (5, 48)).astype(np.float32)
    mean, sd = emri.search_noise_moments(_t(best))
    torch.cuda.synchronize()
    om, osd = osr.noise_moments(best)
    assert np.allclose(_np(mean), om, rtol=1e-14, atol=0)
    assert np.allclose(_np(sd), osd, rtol=1e-12, atol=0)
