"""Solve-serving loop with continuous batching.

Requests ask for solves of Mhat^dag Mhat x = phi (one or more right-hand
sides, each with its own kappa) on one of several resident lattices.  Each
lattice has an executor -- a context with its gauge field and a solver
session (include/wd.h, wd_session_*) on its own HIP stream -- driven by its
own worker thread, so work on different lattices overlaps on the device.

Continuous batching: a worker alternates "admit what fits" and "run k
iterations of every running slot"; requests arriving while others run join
at the next step boundary, and leave as soon as all their right-hand sides
are done.  Admission is FIFO per lattice and by device memory: a session's
slots are allocated when a request needs them (the session grows) and given
back when its lattice's queue drains (it shrinks, or is freed when idle), so
the bytes charged against the global budget -- session slots plus each
request's input/output buffers -- are bytes actually held on the device; each
admission is also checked against the device's free memory.  A lattice with
nothing running whose queue head does not fit gives back its idle slots
before it waits, so idle sessions never hold bytes another lattice's request
needs.

The scheduler core (Admission, Server) is independent of the device: the
executor interface is `max_slots`, `slot_bytes`, `io_bytes(nrhs)`,
`grow_bytes(nrhs)`, `add(req) -> slots`, `step(k)`, `poll() -> states,
stats`, `take(req)` and `shrink() -> bytes freed`.
"""
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

SLOT_FREE, SLOT_RUNNING, SLOT_DONE = 0, 1, 2


@dataclass
class Request:
    rid: int
    lattice: str
    phi: np.ndarray            # [nrhs, Vh, 4, 3] complex128, host
    kappa: list
    arrival: float = 0.0       # seconds after the start of the run
    admitted: float = None
    finished: float = None
    x: np.ndarray = None
    stats: list = field(default_factory=list)
    slots: list = field(default_factory=list)
    nbytes: int = 0

    @property
    def nrhs(self):
        return int(self.phi.shape[0])

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class Admission:
    """Byte budget shared by all lattices.  `free_fn` (optional) returns the
    device's free bytes; a request is admitted only if it fits both."""

    def __init__(self, budget_bytes, free_fn=None, reserve_bytes=0):
        self.budget = int(budget_bytes)
        self.in_use = 0
        self.peak = 0
        self.free_fn = free_fn
        self.reserve = int(reserve_bytes)
        self.lock = threading.Lock()

    def try_take(self, nbytes):
        with self.lock:
            if self.in_use + nbytes > self.budget:
                return False
            if self.free_fn is not None and nbytes + self.reserve > self.free_fn():
                return False
            self.in_use += nbytes
            self.peak = max(self.peak, self.in_use)
            return True

    def give(self, nbytes):
        with self.lock:
            self.in_use -= nbytes
            assert self.in_use >= 0


def percentile(values, q):
    return float(np.percentile(np.asarray(values, dtype=float), q)) if len(values) else float("nan")


class Server:
    """Runs a stream of requests through the executors (one worker thread per
    lattice) and records admission/finish times."""

    def __init__(self, executors, admission, k_iters=8, clock=time.perf_counter):
        self.ex = dict(executors)
        self.adm = admission
        self.k = int(k_iters)
        self.clock = clock
        self.cv = threading.Condition()
        self.queues = {name: deque() for name in self.ex}
        self.t0 = None
        self.closed = False
        self.done = []
        self.errors = []
        self.steps = {name: 0 for name in self.ex}
        self.max_batch = {name: 0 for name in self.ex}

    def now(self):
        return self.clock() - self.t0

    def submit(self, req):
        with self.cv:
            self.queues[req.lattice].append(req)
            self.cv.notify_all()

    def _admit(self, name, running):
        ex = self.ex[name]
        q = self.queues[name]
        used = sum(r.nrhs for r in running)
        while q:
            req = q[0]
            if req.nrhs > ex.max_slots:
                raise ValueError(f"request {req.rid} needs {req.nrhs} slots, lattice {name} has {ex.max_slots}")
            if req.nrhs * ex.slot_bytes + ex.io_bytes(req.nrhs) > self.adm.budget:
                raise ValueError(f"request {req.rid} needs more than the whole budget of {self.adm.budget} bytes")
            if used + req.nrhs > ex.max_slots:
                break
            grow = ex.grow_bytes(req.nrhs)
            io = ex.io_bytes(req.nrhs)
            if not self.adm.try_take(grow + io):
                break
            q.popleft()
            req.nbytes = io
            req.admitted = self.now()
            req.slots = ex.add(req)
            used += req.nrhs
            running.append(req)

    def _worker(self, name):
        ex = self.ex[name]
        running = []
        try:
            while True:
                with self.cv:
                    while True:
                        self._admit(name, running)
                        if running:
                            break
                        if self.closed and not self.queues[name]:
                            self.adm.give(ex.shrink())
                            return
                        if self.queues[name]:
                            # idle, and the queue head does not fit: give back
                            # the idle slots before waiting, or two lattices
                            # that each hold idle slots could wait for each
                            # other's bytes forever
                            freed = ex.shrink()
                            if freed:
                                self.adm.give(freed)
                                self.cv.notify_all()
                                continue
                        self.cv.wait(timeout=0.05)
                self.max_batch[name] = max(self.max_batch[name], sum(r.nrhs for r in running))
                ex.step(self.k)
                self.steps[name] += 1
                states, stats = ex.poll()
                still = []
                finished = False
                for req in running:
                    if all(states[s] == SLOT_DONE for s in req.slots):
                        req.stats = [stats[s] for s in req.slots]
                        req.x = ex.take(req)
                        req.finished = self.now()
                        self.adm.give(req.nbytes)
                        finished = True
                        with self.cv:
                            self.done.append(req)
                    else:
                        still.append(req)
                running = still
                if finished:
                    with self.cv:
                        if not self.queues[name]:
                            # nothing waiting here: return the slots above the
                            # highest one still in use (all of them when idle)
                            self.adm.give(ex.shrink())
                        self.cv.notify_all()
        except Exception as e:  # surfaced by run()
            self.errors.append(e)
            with self.cv:
                self.closed = True
                self.cv.notify_all()

    def run(self, requests, realtime=True):
        """Feed `requests` (sorted by arrival) in real time and wait for all."""
        requests = sorted(requests, key=lambda r: r.arrival)
        self.t0 = self.clock()
        workers = [threading.Thread(target=self._worker, args=(n,), daemon=True) for n in self.ex]
        for w in workers:
            w.start()
        for req in requests:
            if realtime:
                delay = req.arrival - self.now()
                if delay > 0:
                    time.sleep(delay)
            self.submit(req)
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in workers:
            w.join()
        if self.errors:
            raise self.errors[0]
        return self.summary(requests)

    def summary(self, requests):
        lat = [r.latency for r in requests if r.latency is not None]
        makespan = max((r.finished for r in requests if r.finished is not None), default=0.0)
        solves = sum(r.nrhs for r in requests if r.finished is not None)
        return {
            "requests": len(requests),
            "completed": sum(r.finished is not None for r in requests),
            "rhs_solved": solves,
            "makespan_s": makespan,
            "solves_per_s": solves / makespan if makespan > 0 else float("nan"),
            "latency_p50_s": percentile(lat, 50),
            "latency_p99_s": percentile(lat, 99),
            "latency_mean_s": float(np.mean(lat)) if lat else float("nan"),
            "peak_bytes": self.adm.peak,
            "budget_bytes": self.adm.budget,
            "steps": dict(self.steps),
            "max_batch": dict(self.max_batch),
        }


class GpuExecutor:
    """A lattice resident on the GPU: context + gauge field, and a solver
    session that grows to the slots admitted requests need (up to max_slots)
    and shrinks when the scheduler says so; all work on its own stream."""

    def __init__(self, dims, U, params, max_slots, device=0, keep_result=True):
        import torch

        from . import wd
        self.wd = wd
        self.torch = torch
        self.dims = tuple(dims)
        self.Vh = int(np.prod(dims)) // 2
        self.dev = torch.device(f"cuda:{device}")
        self.stream = torch.cuda.Stream(device=self.dev)
        self.max_slots = int(max_slots)
        self.params = params
        with torch.cuda.stream(self.stream):
            self.lat = wd.Lattice(self.dims, device=device, stream=self.stream)
            Ud = torch.from_numpy(np.ascontiguousarray(U)).to(self.dev)
            self.lat.gauge_load(Ud, recon=12)
            self.stream.synchronize()
            del Ud
        self.sess = None
        self.cap = 0
        self.in_use = set()
        self.slot_bytes = wd.wd_session_bytes(self.dims, 1, params)
        self.gauge_bytes = wd.wd_bytes_required(self.dims, 0, params)
        self.bufs = {}
        self.keep_result = keep_result

    def io_bytes(self, nrhs):
        return 2 * nrhs * self.Vh * 192

    def _needed_cap(self, nrhs):
        free = self.cap - len(self.in_use)
        return self.cap + max(0, nrhs - free)

    def grow_bytes(self, nrhs):
        return (self._needed_cap(nrhs) - self.cap) * self.slot_bytes

    def _resize(self, cap):
        if cap == self.cap:
            return
        if cap == 0:
            self.wd.wd_session_destroy(self.sess)
            self.sess = None
        elif self.sess is None:
            self.sess = self.wd.wd_session_create(self.lat.ctx, cap, self.params)
        else:
            self.wd.wd_session_resize(self.sess, cap)
        self.cap = cap

    def add(self, req):
        torch = self.torch
        self._resize(self._needed_cap(req.nrhs))
        with torch.cuda.stream(self.stream):
            if isinstance(req.phi, torch.Tensor):  # a source already on the device
                phi = req.phi.to(self.dev).clone()
            else:
                phi = torch.from_numpy(np.ascontiguousarray(req.phi)).to(self.dev, non_blocking=False)
            x = torch.empty_like(phi)
        self.stream.synchronize()
        slots = self.wd.wd_session_add(self.sess, phi, req.kappa)
        self.in_use.update(slots)
        self.bufs[req.rid] = x
        del phi
        return slots

    def step(self, k):
        self.wd.wd_session_step(self.sess, k)

    def poll(self):
        return self.wd.wd_session_poll(self.sess, self.cap)

    def take(self, req):
        x = self.bufs.pop(req.rid)
        for j, s in enumerate(req.slots):
            self.wd.wd_session_take(self.sess, s, x[j])
            self.in_use.discard(s)
        self.stream.synchronize()
        # keep_result=False drops the solution after it has been unpacked (a
        # throughput measurement that does not collect results)
        return x.cpu().numpy() if self.keep_result else None

    def shrink(self):
        """Free the slots above the highest one in use; returns the bytes."""
        old = self.cap
        self._resize(max(self.in_use) + 1 if self.in_use else 0)
        return (old - self.cap) * self.slot_bytes

    def close(self):
        if self.sess is not None:
            self.wd.wd_session_destroy(self.sess)
            self.sess = None
            self.cap = 0
        self.lat.close()


def poisson_arrivals(n, rate, rng):
    """n arrival times of a Poisson process of the given rate (per second)."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
