"""The serving scheduler on the CPU with a fake executor: every request
completes with its own results (slot reuse), the byte budget and the device's
free memory bound admission, admission is FIFO per lattice, new requests join
running batches (continuous batching), and latencies are accounted."""
import threading
import time

import numpy as np
import pytest

from paper_1207_2223_amd.serve import SLOT_DONE, SLOT_FREE, SLOT_RUNNING, Admission, Request, Server


class FakeExecutor:
    """Slots finish after `need(kappa)` iterations; the 'solution' is 2 phi.
    Like the GPU executor, it holds only the slots it has grown to."""

    def __init__(self, max_slots, slot_bytes=100, step_time=0.002, need_fn=None, held=None):
        self.max_slots = max_slots
        self.need_fn = need_fn or (lambda k: int(round(1000 * k)) % 7 * 8 + 8)
        self.slot_bytes = slot_bytes
        self.step_time = step_time
        self.state, self.count, self.need, self.val = [], [], [], []
        self.max_running = 0
        self.max_cap = 0
        self.held = held if held is not None else {"now": 0, "max": 0}

    @property
    def cap(self):
        return len(self.state)

    def _set_cap(self, cap):
        d = cap - self.cap
        if d > 0:
            self.state += [SLOT_FREE] * d
            self.count += [0] * d
            self.need += [0] * d
            self.val += [None] * d
        else:
            assert all(s == SLOT_FREE for s in self.state[cap:])
            del self.state[cap:], self.count[cap:], self.need[cap:], self.val[cap:]
        self.held["now"] += d * self.slot_bytes
        self.held["max"] = max(self.held["max"], self.held["now"])
        self.max_cap = max(self.max_cap, cap)

    def io_bytes(self, nrhs):
        return 10 * nrhs

    def _missing(self, nrhs):
        return max(0, nrhs - sum(s == SLOT_FREE for s in self.state))

    def grow_bytes(self, nrhs):
        return self._missing(nrhs) * self.slot_bytes

    def add(self, req):
        self._set_cap(self.cap + self._missing(req.nrhs))
        free = [s for s in range(self.cap) if self.state[s] == SLOT_FREE]
        slots = free[:req.nrhs]
        for j, s in enumerate(slots):
            self.state[s] = SLOT_RUNNING
            self.count[s] = 0
            self.need[s] = self.need_fn(req.kappa[j])
            self.val[s] = 2 * req.phi[j]
        self.max_running = max(self.max_running, sum(st != SLOT_FREE for st in self.state))
        return slots

    def step(self, k):
        time.sleep(self.step_time)
        for s in range(self.cap):
            if self.state[s] == SLOT_RUNNING:
                self.count[s] += k
                if self.count[s] >= self.need[s]:
                    self.state[s] = SLOT_DONE

    def poll(self):
        stats = [dict(iters=self.count[s], status=0, true_resid=0.0, reliable_updates=0, seconds=0.0)
                 for s in range(self.cap)]
        return list(self.state), stats

    def take(self, req):
        out = np.stack([self.val[s] for s in req.slots])
        for s in req.slots:
            assert self.state[s] == SLOT_DONE
            self.state[s] = SLOT_FREE
        return out

    def shrink(self):
        used = [s for s in range(self.cap) if self.state[s] != SLOT_FREE]
        old = self.cap
        self._set_cap(max(used) + 1 if used else 0)
        return (old - self.cap) * self.slot_bytes


def make_requests(n, lattices, seed=0, max_nrhs=3, gap=0.001):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        nrhs = int(rng.integers(1, max_nrhs + 1))
        phi = rng.standard_normal((nrhs, 4, 4, 3)) + 1j * rng.standard_normal((nrhs, 4, 4, 3))
        reqs.append(Request(rid=i, lattice=lattices[i % len(lattices)], phi=phi,
                            kappa=list(rng.uniform(0.14, 0.157, nrhs)), arrival=i * gap))
    return reqs


def test_all_complete_with_their_own_results():
    ex = {"a": FakeExecutor(3), "b": FakeExecutor(4)}
    srv = Server(ex, Admission(10 ** 9), k_iters=8)
    reqs = make_requests(20, ["a", "b"])
    summ = srv.run(reqs)
    assert summ["completed"] == 20 and summ["rhs_solved"] == sum(r.nrhs for r in reqs)
    for r in reqs:
        assert np.array_equal(r.x, 2 * r.phi)
        assert r.finished >= r.admitted >= 0
        assert r.latency >= r.finished - r.admitted
    assert ex["a"].max_running <= 3 and ex["b"].max_running <= 4
    assert summ["latency_p99_s"] >= summ["latency_p50_s"] > 0
    # every slot is given back once the stream has drained
    assert ex["a"].cap == 0 and ex["b"].cap == 0 and srv.adm.in_use == 0


def test_budget_bounds_admission_and_fifo_order():
    ex = {"a": FakeExecutor(8)}
    # every request costs nrhs*100 + nrhs*10 bytes; a budget of 330 admits at most 3 RHS
    adm = Admission(330)
    srv = Server(ex, adm, k_iters=8)
    reqs = make_requests(12, ["a"], max_nrhs=3)
    srv.run(reqs)
    assert adm.peak <= 330 and adm.in_use == 0
    assert ex["a"].max_running <= 3
    adm_order = sorted(reqs, key=lambda r: r.admitted)
    assert [r.rid for r in adm_order] == sorted(r.rid for r in reqs)  # FIFO


def test_free_memory_bounds_admission():
    # a device with 250 free bytes that the admitted requests use up
    adm = Admission(10 ** 9)
    adm.free_fn = lambda: 250 - adm.in_use
    ex = {"a": FakeExecutor(8)}
    srv = Server(ex, adm, k_iters=8)
    reqs = make_requests(6, ["a"], max_nrhs=2)
    srv.run(reqs)
    # with 250 free bytes at most 2 RHS (220 bytes) fit at a time
    assert ex["a"].max_running <= 2


def test_budget_is_shared_by_lattices_and_counts_held_slots():
    # 3 slots' worth of budget (plus io) shared by two lattices: the slots the
    # two sessions hold together never exceed it, and both make progress
    held = {"now": 0, "max": 0}
    ex = {"a": FakeExecutor(4, held=held), "b": FakeExecutor(4, held=held)}
    adm = Admission(3 * 100 + 3 * 10)
    srv = Server(ex, adm, k_iters=8)
    reqs = make_requests(16, ["a", "b"], max_nrhs=2, seed=3)
    summ = srv.run(reqs)
    assert summ["completed"] == 16
    assert held["max"] <= 300 and held["now"] == 0
    assert adm.peak <= 330 and adm.in_use == 0
    assert ex["a"].max_cap >= 1 and ex["b"].max_cap >= 1


def test_continuous_batching_joins_running_batch():
    ex = {"a": FakeExecutor(4, step_time=0.01, need_fn=lambda k: 400 if k > 0.155 else 8)}
    srv = Server(ex, Admission(10 ** 9), k_iters=8)
    phi = np.ones((1, 4, 4, 3), complex)
    long_req = Request(0, "a", phi, [0.1556], arrival=0.0)   # needs many iterations
    late_req = Request(1, "a", 3 * phi, [0.15], arrival=0.03)
    srv.run([long_req, late_req])
    assert late_req.admitted < long_req.finished
    assert np.array_equal(late_req.x, 6 * phi)


def test_oversized_request_is_an_error():
    ex = {"a": FakeExecutor(2)}
    srv = Server(ex, Admission(10 ** 9), k_iters=8)
    bad = Request(0, "a", np.zeros((3, 4, 4, 3), complex), [0.15] * 3)
    with pytest.raises(ValueError):
        srv.run([bad])


def test_latency_accounting_with_arrivals():
    ex = {"a": FakeExecutor(3, step_time=0.002)}
    srv = Server(ex, Admission(10 ** 9), k_iters=8)
    reqs = make_requests(8, ["a"], gap=0.01)
    summ = srv.run(reqs)
    for r in reqs:
        assert r.admitted >= r.arrival - 1e-3
    lat = sorted(r.latency for r in reqs)
    assert abs(summ["latency_p50_s"] - float(np.percentile(lat, 50))) < 1e-12


def test_idle_slots_are_released_when_two_lattices_block_each_other():
    # Two lattices each finish a 2-RHS request and keep 2 idle slots while
    # their next requests (3 RHS each) wait.  The budget (4 slots plus io)
    # fits one 3-RHS request at a time only if the other lattice's idle slots
    # are given back; otherwise both heads would wait for each other forever.
    ex = {"a": FakeExecutor(4, step_time=0.002), "b": FakeExecutor(4, step_time=0.002)}
    adm = Admission(4 * 100 + 4 * 10)
    srv = Server(ex, adm, k_iters=8)
    phi2, phi3 = np.ones((2, 4, 4, 3), complex), np.ones((3, 4, 4, 3), complex)
    reqs = [Request(0, "a", phi2, [0.15, 0.15], arrival=0.0),
            Request(1, "b", phi2, [0.15, 0.15], arrival=0.0),
            Request(2, "a", 2 * phi3, [0.15] * 3, arrival=0.001),
            Request(3, "b", 3 * phi3, [0.15] * 3, arrival=0.001)]
    out = {}
    th = threading.Thread(target=lambda: out.update(summ=srv.run(reqs)), daemon=True)
    th.start()
    th.join(timeout=20)
    assert not th.is_alive(), "scheduler deadlocked"
    assert out["summ"]["completed"] == 4
    for r in reqs:
        assert np.array_equal(r.x, 2 * r.phi)
    assert adm.peak <= 440 and adm.in_use == 0


@pytest.mark.parametrize("seed", range(60))
def test_random_streams_complete_within_a_tight_budget(seed):
    """Random streams (2-4 lattices of different slot sizes, 1-8 RHS per
    request, Poisson arrivals) under a budget that fits the largest request
    alone plus at most 300 bytes: every request completes with its own
    results, the budget is never exceeded and everything is given back."""
    rng = np.random.default_rng(seed)
    nl = int(rng.integers(2, 5))
    sb = {f"L{i}": int(rng.choice([50, 100, 200])) for i in range(nl)}
    ex = {k: FakeExecutor(8, slot_bytes=v, step_time=0.0005) for k, v in sb.items()}
    budget = max(8 * v + 80 for v in sb.values()) + int(rng.integers(0, 300))
    adm = Admission(budget)
    srv = Server(ex, adm, k_iters=8)
    reqs, t = [], 0.0
    for i in range(16):
        n = int(rng.integers(1, 9))
        t += float(rng.exponential(0.002))
        reqs.append(Request(i, f"L{int(rng.integers(nl))}", rng.standard_normal((n, 4, 4, 3)) + 0j,
                            list(rng.uniform(0.14, 0.157, n)), arrival=t))
    out = {}
    th = threading.Thread(target=lambda: out.update(summ=srv.run(reqs)), daemon=True)
    th.start()
    th.join(timeout=30)
    assert not th.is_alive(), f"scheduler stalled (budget {budget}, slot bytes {sb})"
    assert out["summ"]["completed"] == len(reqs)
    for r in reqs:
        assert np.array_equal(r.x, 2 * r.phi)
    assert adm.peak <= budget and adm.in_use == 0
