"""Continuous-batching server for PMACE reconstructions.

Requests (one ptychography problem each) arrive over time.  The server keeps
every admitted reconstruction's agent states resident on the GPU, admits new
requests as soon as their workspace fits in the memory budget and a slot is
free, advances all active reconstructions together (one batched graph launch
per iteration, stop rule evaluated on the device), and retires each as soon as
it has converged, copying its reconstruction back.  The same executor run with
one request at a time, in arrival order, is the plain solver it is compared
with.

The executor interface keeps the scheduling logic testable without a GPU:

    footprint(problem) -> bytes      workspace a request will hold while active
    work(problem) -> float           work per iteration (patch pixels), for the
                                     size-class policy (optional)
    admit(req)                       start a reconstruction (device state resident)
    step(n)                          n iterations of every active reconstruction
    poll() -> {req_id: (done, nrmse, iters)}
    retire(req_id) -> result         reconstruction back to the host, memory freed
"""
from __future__ import annotations

import dataclasses
import heapq
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    problem: object            # a synth.Problem (or anything the executor understands)
    arrival: float             # seconds since the start of the run
    admitted: Optional[float] = None
    finished: Optional[float] = None
    iters: int = 0
    nrmse: float = float("nan")
    result: object = None
    x0: object = None          # starting object (None: the default start, 1 everywhere)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class WallClock:
    """Real time since construction; sleep() waits."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        d = t - self.now()
        if d > 0:
            time.sleep(d)


class FakeClock:
    """Deterministic clock for tests: time advances only when told to."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def advance(self, dt: float):
        self.t += dt

    def sleep_until(self, t: float):
        self.t = max(self.t, t)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process (exponential inter-arrival times)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


@dataclasses.dataclass
class ServeStats:
    completed: int
    makespan: float
    solves_per_s: float
    p50: float
    p99: float
    mean_latency: float
    max_active: int
    steps: int
    host_s: Optional[Dict[str, float]] = None   # wall time inside admit / step / poll / retire

    def as_dict(self):
        return dataclasses.asdict(self)


def _stats(reqs: Sequence[Request], makespan: float, max_active: int, steps: int,
           host_s: Optional[Dict[str, float]] = None) -> ServeStats:
    lat = np.array([r.latency for r in reqs if r.finished is not None])
    return ServeStats(completed=len(lat), makespan=makespan,
                      solves_per_s=len(lat) / makespan if makespan > 0 else float("nan"),
                      p50=float(np.percentile(lat, 50)) if len(lat) else float("nan"),
                      p99=float(np.percentile(lat, 99)) if len(lat) else float("nan"),
                      mean_latency=float(lat.mean()) if len(lat) else float("nan"),
                      max_active=max_active, steps=steps, host_s=host_s)


class Server:
    """Continuous batching: admit on arrival when memory and a slot allow,
    step every active reconstruction together, retire each on convergence.

    capacity_bytes  memory budget for the workspaces of active requests
    max_active      upper bound on concurrently active requests
    iters_per_step  iterations launched between polls of the stop flags
    on_step         optional hook(clock, n_active, iters) after each step (a
                    fake clock advances there in tests)
    large_work      size-class policy: a request whose work per iteration is
                    at least this is "large"; at most max_large large requests
                    are active at once (FIFO among them), while smaller
                    requests are admitted past a waiting large one.  Sharing
                    the device equally would stretch a large request by the
                    work of everything admitted during its lifetime; this
                    keeps large requests close to their solo time and small
                    ones from queueing behind them.  None: one class.
    hold_small      with size classes: while a large request waits for the
                    large slot, smaller ones are not admitted either (the
                    running large request then shares the device with fewer
                    others and the large queue drains sooner).
    """

    def __init__(self, executor, capacity_bytes: int, max_active: int = 64,
                 iters_per_step: int = 4, on_step: Optional[Callable] = None,
                 large_work: Optional[float] = None, max_large: int = 1,
                 hold_small: bool = False):
        self.ex = executor
        self.capacity = int(capacity_bytes)
        self.max_active = int(max_active)
        self.iters_per_step = int(iters_per_step)
        self.on_step = on_step
        self.large_work = large_work
        self.max_large = int(max_large)
        self.hold_small = bool(hold_small)

    def _large(self, req) -> bool:
        return self.large_work is not None and self.ex.work(req.problem) >= self.large_work

    def run(self, requests: List[Request], clock) -> ServeStats:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if self.ex.footprint(r.problem) > self.capacity:
                raise ValueError(f"request {r.rid} needs more memory than the whole budget")
        queue: List[Request] = []          # arrived, not admitted (FIFO)
        active: Dict[int, Request] = {}
        used = 0
        n_large = 0
        nxt = 0
        max_active = 0
        steps = 0
        host = {"admit": 0.0, "step": 0.0, "poll": 0.0, "retire": 0.0}
        tick = time.perf_counter
        while nxt < len(pending) or queue or active:
            now = clock.now()
            while nxt < len(pending) and pending[nxt].arrival <= now:
                queue.append(pending[nxt])
                nxt += 1
            # launch the next iterations of the active requests first, so the
            # host-side set-up of new admissions overlaps them on the device
            stepped = bool(active)
            if stepped:
                t0 = tick()
                self.ex.step(self.iters_per_step)
                host["step"] += tick() - t0
                steps += 1
                if self.on_step:
                    self.on_step(clock, len(active), self.iters_per_step)
            # admission in arrival order while memory and slots allow; a large
            # request waiting for the large slot does not block smaller ones
            i = 0
            large_waiting = False
            while i < len(queue) and len(active) < self.max_active:
                r = queue[i]
                fp = self.ex.footprint(r.problem)
                if used + fp > self.capacity:
                    break
                large = self._large(r)
                if large and n_large >= self.max_large:
                    large_waiting = True
                    i += 1
                    continue
                if not large and large_waiting and self.hold_small:
                    break
                queue.pop(i)
                t0 = tick()
                self.ex.admit(r)
                host["admit"] += tick() - t0
                r.admitted = clock.now()
                active[r.rid] = r
                used += fp
                n_large += int(large)
            max_active = max(max_active, len(active))
            if not stepped:
                if not active and nxt < len(pending):
                    clock.sleep_until(pending[nxt].arrival)
                continue
            t1 = tick()
            polled = self.ex.poll()
            host["poll"] += tick() - t1
            for rid, (done, nr, it) in polled.items():
                if not done:
                    continue
                r = active.pop(rid)
                t0 = tick()
                r.result = self.ex.retire(rid)
                host["retire"] += tick() - t0
                r.finished = clock.now()
                r.iters, r.nrmse = int(it), float(nr)
                used -= self.ex.footprint(r.problem)
                n_large -= int(self._large(r))
        makespan = clock.now() - (pending[0].arrival if pending else 0.0)
        return _stats(requests, makespan, max_active, steps, host)


def run_plain(executor, requests: List[Request], clock, iters_per_step: int = 4,
              on_step: Optional[Callable] = None) -> ServeStats:
    """The plain solver: one request at a time, in arrival order, to convergence."""
    srv = Server(executor, capacity_bytes=1 << 62, max_active=1, iters_per_step=iters_per_step,
                 on_step=on_step)
    return srv.run(requests, clock)


class GPUExecutor:
    """Executor on the HIP library: one Reconstruction (device-resident state)
    per active request, re-batched whenever the active set changes.

    split_work: requests with at least this much work per iteration (patch
    pixels) are stepped in a batch and on a stream of their own, so the churn
    of small requests (each admission or retirement rebuilds a batch, and a
    rebuilt batch runs uncaptured for its first steps) leaves the large
    requests' batch, and its captured graph, alone; the two batches advance
    concurrently.  None: one batch for everything."""

    def __init__(self, alpha: float, kappa: float = 1.25, rho: float = 0.5, tol: float = 1e-4,
                 min_iter: int = 2, max_iter: int = 500, device="cuda", stream=None,
                 criterion: int = 0, check_every: int = 1, split_work: Optional[float] = None):
        from . import pmace, synth
        self._pmace = pmace
        self._synth = synth
        self.alpha, self.kappa, self.rho = alpha, kappa, rho
        self.tol, self.min_iter, self.max_iter = tol, min_iter, max_iter
        self.criterion, self.check_every = criterion, check_every
        self.device = device
        self.split_work = split_work
        self.active: Dict[int, object] = {}
        self._fp_cache: Dict[tuple, int] = {}
        import torch
        self._torch = torch
        # new reconstructions are set up on a side stream, so their host work
        # and synchronisations overlap the running batches
        self.init_stream = torch.cuda.Stream(device=device)
        streams = [stream, torch.cuda.Stream(device=device) if split_work is not None else stream]
        # group 0: all requests (or the small ones), group 1: the large ones
        self.groups = [{"order": [], "batch": None, "dirty": False, "stream": st, "batch_order": []}
                       for st in streams]
        self.group_of: Dict[int, int] = {}

    def footprint(self, prob) -> int:
        """Device bytes a request holds while active: its workspace, its NRMSE
        reference and region (8 + 1 B per object pixel), the reconstruction
        copied out at retirement (8 B per pixel), and a bound on its share of
        a batch workspace (descriptor, work items, gather items, reduction
        items)."""
        key = (prob.n1, prob.n2, prob.np_, prob.num_pos)
        if key not in self._fp_cache:
            prm = self._pmace.make_params(prob.n1, prob.n2, prob.np_, prob.num_pos, self.alpha,
                                          self.kappa, self.rho)
            npx = prob.n1 * prob.n2
            batch_share = 1024 + 8 * prob.num_pos + npx // 16 + 8 * (npx // 4096 + 1)
            self._fp_cache[key] = self._pmace.pmace_footprint(prm) + 17 * npx + batch_share
        return self._fp_cache[key]

    def work(self, prob) -> float:
        return float(prob.num_pos) * prob.np_ * prob.np_

    def admit(self, req):
        p = req.problem
        gi = int(self.split_work is not None and self.work(p) >= self.split_work)
        g = self.groups[gi]
        with self._torch.cuda.stream(self.init_stream):
            R = self._pmace.Reconstruction(p.n1, p.n2, p.probe, p.pos, p.z, self.alpha, self.kappa,
                                           self.rho, x0=req.x0, device=self.device,
                                           stream=self.init_stream)
            R.set_reference(p.x_true, self._synth.roi_mask(p.probe, p.pos, p.n1, p.n2))
        R.set_stream(g["stream"])
        self.active[req.rid] = R
        self.group_of[req.rid] = gi
        g["order"].append(req.rid)
        g["dirty"] = True            # joins its group's batch at the next step

    @staticmethod
    def _drop(g):
        if g["batch"] is not None:
            g["batch"].close()
            g["batch"] = None

    def step(self, n: int):
        for g in reversed(self.groups):      # the large requests' batch is launched first
            if g["dirty"]:
                self._drop(g)
                g["dirty"] = False
            if not g["order"]:
                continue
            if g["batch"] is None:           # membership changed since the last step
                g["batch_order"] = list(g["order"])
                g["batch"] = self._pmace.Batch([self.active[r] for r in g["order"]], tol=self.tol,
                                               min_iter=self.min_iter, max_iter=self.max_iter,
                                               criterion=self.criterion, check_every=self.check_every)
            g["batch"].step(n)
            if self.split_work is None:
                break

    def poll(self):
        out = {}
        for g in self.groups:
            if g["batch"] is None:
                continue
            done, nr, it = g["batch"].poll()
            # members admitted since the last step are not in the batch yet
            out.update({rid: (bool(done[i]), float(nr[i]), int(it[i]))
                        for i, rid in enumerate(g["batch_order"])})
            if self.split_work is None:
                break
        return out

    def retire(self, rid):
        R = self.active.pop(rid)
        g = self.groups[self.group_of.pop(rid)]
        with self._torch.cuda.stream(g["stream"]):   # the copy follows R's own work
            x = R.reconstruct().cpu().numpy()
        self._drop(g)                # the batch reads R's descriptor: release it first
        g["order"].remove(rid)
        R.close()
        return x
