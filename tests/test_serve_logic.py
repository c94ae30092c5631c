"""Scheduling logic of the continuous-batching server, on a fake backend (no GPU)."""
import numpy as np
import pytest

from paper_2310_17790_amd.serve import Request, Server


class FakeSim:
    def __init__(self, w):
        self.w = w
        self.steps = 0


class FakeBackend:
    """Sims are step counters; a step of a batch costs 1 ms per member."""

    def __init__(self):
        self.ticks = []
        self.created = []

    def sim_bytes(self, w):
        return int(w.X.shape[1]) * 100

    def create(self, w):
        self.created.append(w.rid)
        return FakeSim(w)

    def step(self, sims):
        for s in sims:
            s.steps += 1
        self.ticks.append(float(len(sims)))

    def tick_ms(self):
        return list(self.ticks)

    def wait_behind(self, depth):
        pass

    def finish(self, sim, keep):
        return np.array([float(sim.steps)]), 0, None


class W:
    def __init__(self, rid, n):
        self.rid = rid
        self.X = np.zeros((3, n))


class StepClock:
    """Deterministic clock: advances 1 ms per reading."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


def _requests():
    rng = np.random.default_rng(0)
    t = np.cumsum(rng.exponential(0.005, size=20))
    return [Request(i, float(t[i]), W(i, int(rng.integers(50, 500))), steps=int(rng.integers(5, 40)))
            for i in range(20)]


def test_all_requests_complete_with_their_steps():
    be = FakeBackend()
    srv = Server(be, hbm_budget_bytes=100_000, clock=StepClock())
    reqs = _requests()
    srv.submit(reqs)
    st = srv.run()
    assert st["requests"] == 20
    got = {r.rid: r for r in srv.results}
    for q in reqs:
        assert got[q.rid].steps == q.steps
        assert got[q.rid].z[0] == q.steps          # the sim advanced exactly its own steps
    assert st["latent_steps"] == sum(q.steps for q in reqs)


def test_budget_and_fifo_admission():
    be = FakeBackend()
    budget = 60_000
    srv = Server(be, hbm_budget_bytes=budget, clock=StepClock())
    reqs = _requests()
    srv.submit(reqs)
    srv.run()
    assert srv.peak_used <= budget
    # admitted strictly in arrival order
    order = [q.rid for q in sorted(reqs, key=lambda q: q.arrival_s)]
    assert be.created == order
    # the budget forced queueing: some request waited after arriving
    assert any(r.admitted_s > r.arrival_s + 1e-3 for r in srv.results)


def test_continuous_batching_changes_membership_mid_run():
    be = FakeBackend()
    srv = Server(be, hbm_budget_bytes=10 ** 9, clock=StepClock())
    srv.submit(_requests())
    srv.run()
    sizes = [t["n"] for t in srv.ticks]
    # sims join while others run and leave while others continue
    assert max(sizes) > 1
    assert any(b > a for a, b in zip(sizes, sizes[1:]))
    assert any(b < a for a, b in zip(sizes, sizes[1:]))


def test_slot_limit():
    be = FakeBackend()
    srv = Server(be, hbm_budget_bytes=10 ** 9, max_slots=3, clock=StepClock())
    srv.submit(_requests())
    srv.run()
    assert srv.peak_active <= 3


def test_request_larger_than_budget_is_rejected():
    be = FakeBackend()
    srv = Server(be, hbm_budget_bytes=1000, clock=StepClock())
    srv.submit([Request(0, 0.0, W(0, 500), steps=3)])
    with pytest.raises(ValueError):
        srv.run()
