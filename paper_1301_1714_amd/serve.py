"""Continuous-batching server of DEM solve requests.

A request is one independent system and a number of time steps.  Requests
that have arrived wait in FIFO order; at every iteration the server admits
from the head of the queue as many as fit both a slot limit and an HBM budget
(the workspace bytes of the group they would form), starts them as one group
(one batched engine on its own stream, its state resident on the device until
the request retires), steps every live group by one chunk, and retires the
requests whose steps are done.  Groups run concurrently on their streams, so
requests that arrive while others run are admitted as soon as memory and
slots allow and their work overlaps with the running ones.

A group whose members finish at different times is compacted at the chunk
boundary after a member finishes: the survivors' exact state (positions,
velocities, spins, last forces and tangential history) is read back and a
new, smaller group is built from it, so that the finished members' memory and
slots go back to the pool while the others run on (a restart from that state
is bitwise the uninterrupted run).

A system's arithmetic does not depend on its group or on how its steps are
chunked, so a request's result is the same as the system stepped alone.  If a
group fails (a contact-list overflow, a particle out of the domain, a
non-finite force), each of its unfinished requests is restarted alone from its
initial state, so that only the request at fault fails.

The executor is pluggable: ``GpuExecutor`` (the product path) drives
``dem.Batch``; tests drive the same scheduler with a CPU stand-in.
"""
import math
import time
from collections import deque

import numpy as np


class Request:
    def __init__(self, rid, system, steps, arrival):
        self.rid = rid
        self.system = system      # dict: params, x, v, omega, r
        self.steps = int(steps)
        self.arrival = float(arrival)
        self.t_admit = None
        self.t_done = None
        self.result = None        # read_state() of the finished system
        self.error = None
        self.restarts = 0

    @property
    def n(self):
        return len(self.system["r"])

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class GpuExecutor:
    """Groups are ``dem.Batch`` objects on their own streams, replaying each
    step from HIP graphs."""

    def __init__(self, use_graph=True):
        from . import dem

        self.dem = dem
        self.use_graph = use_graph
        self.errors = (dem.DemError,)

    def workspace_bytes(self, systems):
        return self.dem.dem_batch_workspace_bytes([s["params"] for s in systems], [len(s["r"]) for s in systems])

    def start(self, systems):
        import torch

        st = torch.cuda.Stream()
        b = self.dem.Batch(systems, stream=st)
        if self.use_graph:
            b.use_graph(True)
        return b

    def free_bytes(self):
        import torch

        return torch.cuda.mem_get_info()[0]

    def run_alone(self, system, steps, use_graph=False):
        """The plain single-system path: create, step, read back."""
        import torch

        st = torch.cuda.Stream() if use_graph else None
        s = self.dem.System(system["params"], system["x"], system["v"], system["omega"], system["r"], stream=st)
        try:
            if use_graph:
                s.use_graph(True)
            s.step(steps)
            return s.read_state()
        finally:
            s.close()


class _Group:
    def __init__(self, handle, members, nbytes):
        self.handle = handle
        self.members = members
        self.left = [m.steps for m in members]
        self.bytes = nbytes


class Server:
    """The scheduler.  hbm_budget: bytes the live groups may hold together;
    max_slots: systems resident at once; chunk: steps per iteration."""

    def __init__(self, executor, hbm_budget, max_slots=64, chunk=100, clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.clock = clock
        self.sleep = sleep
        self.iterations = 0
        self.peak_bytes = 0
        self.peak_slots = 0
        self.compactions = 0

    def run(self, requests):
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting = deque()
        live = []
        used = 0
        slots = 0
        done = []
        t0 = self.clock()
        while pending or waiting or live:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission from the head of the queue
            new = []
            nbytes = 0
            while waiting and slots + len(new) < self.max_slots:
                head = waiting[0]
                if head.restarts and new:
                    break  # a restarted request runs alone
                b = self.ex.workspace_bytes([r.system for r in new + [head]])
                if used + b > self.budget:
                    break
                new.append(waiting.popleft())
                nbytes = b
                if head.restarts:
                    break
            if not new and not live and waiting:
                # the head does not fit even on an idle device
                r = waiting.popleft()
                r.error = "workspace larger than the HBM budget"
                r.t_done = self.clock() - t0
                done.append(r)
                continue
            if new:
                live.append(self._start(new, nbytes, t0))
                used += nbytes
                slots += len(new)
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_slots = max(self.peak_slots, slots)
            if not live:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            # one chunk on every live group: launch all, then wait for each
            failed = {}
            for g in live:
                try:
                    g.handle.step([min(self.chunk, l) for l in g.left])
                except self.ex.errors as e:
                    failed[id(g)] = e
            self.iterations += 1
            keep = []
            for g in live:
                err = failed.get(id(g))
                if err is None:
                    try:
                        g.handle.sync()
                    except self.ex.errors as e:
                        err = e
                if err is not None:
                    g.handle.close()
                    used -= g.bytes
                    slots -= len(g.members)
                    retry = []
                    for m, l in zip(g.members, g.left):
                        if l == 0:
                            continue
                        if len(g.members) == 1:
                            m.error = str(err)
                            m.t_done = self.clock() - t0
                            done.append(m)
                        else:
                            m.restarts += 1
                            retry.append(m)
                    waiting.extendleft(reversed(retry))
                    continue
                g.left = [max(0, l - self.chunk) for l in g.left]
                finished = 0
                for k, (m, l) in enumerate(zip(g.members, g.left)):
                    if l == 0 and m.result is None:
                        m.result = g.handle.read_state(k)
                        m.t_done = self.clock() - t0
                        done.append(m)
                        finished += 1
                if all(l == 0 for l in g.left):
                    g.handle.close()
                    used -= g.bytes
                    slots -= len(g.members)
                elif finished:
                    ng = self._compact(g)
                    used += ng.bytes - g.bytes
                    slots -= len(g.members) - len(ng.members)
                    keep.append(ng)
                else:
                    keep.append(g)
            live = keep
        return done

    def _compact(self, g):
        """A new group of g's unfinished members, started from their exact
        current state; g is closed."""
        systems, members, left = [], [], []
        for k, (m, l) in enumerate(zip(g.members, g.left)):
            if l == 0:
                continue
            st = g.handle.read_state(k)
            pairs, dts = g.handle.read_contacts(k)
            systems.append(dict(m.system, x=st["x"], v=st["v"], omega=st["omega"], F=st["F"], T=st["T"],
                                hist_pairs=pairs, hist_dt=dts))
            members.append(m)
            left.append(l)
        nbytes = self.ex.workspace_bytes(systems)
        g.handle.close()
        ng = _Group(self.ex.start(systems), members, nbytes)
        ng.left = left
        self.compactions += 1
        return ng

    def _start(self, members, nbytes, t0):
        handle = self.ex.start([m.system for m in members])
        t = self.clock() - t0
        for m in members:
            m.t_admit = t
        return _Group(handle, members, nbytes)


def one_at_a_time(executor_run, requests):
    """Service time of each request run alone (``executor_run(request)``
    returns its result), in arrival order."""
    service = []
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        t0 = time.perf_counter()
        executor_run(r)
        service.append(time.perf_counter() - t0)
    return np.array(service)


def fifo_latencies(arrivals, service):
    """Completion latencies of a single FIFO server with the given arrival
    and service times (the one-at-a-time baseline on the same arrivals)."""
    t = 0.0
    out = []
    for a, s in zip(arrivals, service):
        start = max(t, a)
        t = start + s
        out.append(t - a)
    return np.array(out)


def percentiles(lat):
    lat = np.asarray(lat, float)
    if lat.size == 0:
        return {"p50": None, "p99": None, "mean": None}
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "mean": float(lat.mean())}


def particle_steps(requests):
    return float(sum(r.n * r.steps for r in requests))


def rate_for_load(load, busy_throughput, mean_work):
    """Arrival rate that keeps a server of the given throughput (particle-
    steps/s) busy the fraction `load` of the time, for requests of mean work
    mean_work particle-steps."""
    return load * busy_throughput / mean_work if mean_work > 0 else math.inf
