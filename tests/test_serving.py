"""Request loop of the serving form, on the CPU with a fake executor:
admission by the HBM budget in arrival order, continuous batching into free
slots, batch limits, completion and latency bookkeeping."""
import numpy as np
import pytest

from paper_2510_20891_amd.serving import Request, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a batch `delay` seconds after launch; the 'top-k' of a request is its row sums."""

    def __init__(self, clock, slots, delay):
        self.clock, self.delay = clock, delay
        self.due = [None] * slots
        self.reqs = [None] * slots
        self.launches = []

    def launch(self, slot, reqs):
        assert self.due[slot] is None
        self.due[slot] = self.clock() + self.delay
        self.reqs[slot] = reqs
        self.launches.append((slot, [r.rid for r in reqs], self.clock()))

    def poll(self, slot):
        if self.due[slot] is None or self.clock() < self.due[slot]:
            return False
        for r in self.reqs[slot]:
            s = r.coeffs.sum(axis=1)
            order = np.lexsort((np.arange(r.n), -s))[: r.top_k]
            r.topk_val, r.topk_idx = s[order], order
        self.due[slot] = self.reqs[slot] = None
        return True


def make_requests(n, K=8, seed=0, rate=2000.0):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, n))
    sizes = np.floor(np.exp(g.uniform(np.log(256), np.log(65536), n))).astype(int)
    return [Request(i, int(g.integers(0, 16)), g.standard_normal((int(m), K)).astype(np.float32), 32, float(ti))
            for i, (ti, m) in enumerate(zip(t, sizes))]


def drive(server, clock, reqs, dt=1e-4):
    pending = sorted(reqs, key=lambda r: r.t_arrival)
    i = 0
    while i < len(pending) or server.busy():
        while i < len(pending) and pending[i].t_arrival <= clock.t:
            server.submit(pending[i])
            i += 1
        server.step()
        assert server.used_bytes <= server.hbm_budget
        clock.t += dt


def test_every_request_served_within_budget_and_limits():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=2, delay=1e-3)
    budget = 8 << 20
    srv = Server(ex, 8, hbm_budget=budget, max_batch_templates=1 << 17, max_requests=64, slots=2, clock=clock)
    reqs = make_requests(400)
    drive(srv, clock, reqs)
    assert len(srv.done) == 400 and srv.used_bytes == 0
    for slot, rids, t in ex.launches:
        batch = [reqs[i] for i in rids]
        assert len(batch) <= 64
        assert sum((r.n + 3) // 4 * 4 for r in batch) <= (1 << 17) or len(batch) == 1
    # admission in arrival order
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.t_arrival)]
    assert all(a <= b for a, b in zip(admits, admits[1:]))
    for r in reqs:
        assert r.t_arrival <= r.t_admit <= r.t_done
        s = r.coeffs.sum(axis=1)
        assert np.array_equal(r.topk_idx, np.lexsort((np.arange(r.n), -s))[:32])


def test_continuous_batching_fills_free_slots_while_others_run():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=3, delay=5e-3)
    srv = Server(ex, 8, hbm_budget=1 << 30, max_batch_templates=1 << 20, max_requests=256, slots=3, clock=clock)
    reqs = make_requests(300, seed=1, rate=20000.0)
    drive(srv, clock, reqs)
    # overlapping launches: a slot launched while another was still running
    busy_overlap = any(abs(t1 - t0) < 5e-3 and s0 != s1
                       for (s0, _, t0), (s1, _, t1) in zip(ex.launches, ex.launches[1:]))
    assert busy_overlap
    assert max(len(r) for _, r, _ in ex.launches) > 1          # requests were batched together
    st = srv.stats(reqs)
    assert st.n_requests == 300 and st.latency_ms["p50"] >= 5.0 - 1e-6


def test_budget_blocks_then_releases():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=2, delay=2e-3)
    one = Request(0, 0, np.zeros((1000, 8), np.float32), 32, 0.0)
    budget = 2 * one.device_bytes(8) + 10          # two such requests at a time
    srv = Server(ex, 8, hbm_budget=budget, max_batch_templates=4096, max_requests=8, slots=2, clock=clock)
    reqs = [Request(i, 0, np.zeros((1000, 8), np.float32), 32, 0.0) for i in range(6)]
    for r in reqs:
        srv.submit(r)
    srv.step()
    assert len(srv.waiting) == 4 and srv.used_bytes == 2 * one.device_bytes(8)
    drive(srv, clock, [])
    assert len(srv.done) == 6


def test_request_that_can_never_fit_is_rejected():
    clock = FakeClock()
    srv = Server(FakeExecutor(clock, 1, 1e-3), 8, hbm_budget=1 << 20, max_batch_templates=1 << 10,
                 max_requests=4, slots=1, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(Request(0, 0, np.zeros((2048, 8), np.float32), 32, 0.0))
