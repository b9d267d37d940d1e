"""Continuous-batching request loop for long-range evaluations.

Requests (one structure each: positions, per-channel charges, box, channel
exponents) arrive over time.  The scheduler keeps several evaluations in
flight on separate HIP streams, so requests that arrive while others run are
admitted as soon as a slot is free and their HBM footprint (workspace +
inputs + outputs) fits the budget, and their work overlaps on the device.
Plans (the per-box host set-up, a fraction of a millisecond once the
shared host caches are warm) are built as requests arrive: inline by
default, or on a worker pool (plan_workers > 0) -- Python threads share one
interpreter lock, which can delay the scheduling loop by its switch
interval, so the pool only pays when plan building is slow.  Each request's result does not depend on
what else is in flight: every kernel works on one structure's own buffers
and all reductions have a fixed order.

The scheduler is written against a small executor interface so that its
admission logic is exercised on the CPU with a simulated executor
(tests/test_serving_cpu.py) and on the GPU with HipExecutor.
"""
import collections
import concurrent.futures
import dataclasses
import gc
import time
from typing import Any, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    pos: np.ndarray            # float32 [N, 3]
    q: np.ndarray              # float32 [C, N]
    box: tuple
    ps: tuple
    t_arrival: float = 0.0     # seconds on the server clock
    # filled by the server
    t_ready: Optional[float] = None
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    energy: Optional[np.ndarray] = None
    forces: Optional[np.ndarray] = None
    virial: Optional[np.ndarray] = None
    error: Optional[str] = None
    footprint: int = 0

    @property
    def n_atoms(self):
        return int(self.pos.shape[0])

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class HipExecutor:
    """Runs requests through the C ABI on per-slot HIP streams."""

    def __init__(self, slots=4, r_c=5.0, c=0.0, tol=1e-5, support=8, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.r_c, self.c, self.tol, self.support = r_c, c, tol, support
        # per-slot pinned staging, grown geometrically and reused: a slot
        # takes a new request only after the previous one's copies are done,
        # and no request pays a pinned allocation
        self._pinned = [dict() for _ in range(slots)]

    def reserve(self, n_atoms, n_channels):
        """Allocate every slot's pinned staging for requests of up to
        n_atoms atoms and n_channels channels ahead of serving."""
        torch = self.torch
        for slot in range(self.slots):
            self._stage(slot, "pos", (n_atoms, 3), torch.float32)
            self._stage(slot, "q", (n_channels, n_atoms), torch.float32)
            self._stage(slot, "energy", (3 * n_channels + 1,), torch.float64)
            self._stage(slot, "forces", (n_atoms, 3), torch.float32)
            self._stage(slot, "virial", (6,), torch.float64)

    def _stage(self, slot, name, shape, dtype):
        n = 1
        for d in shape:
            n *= d
        buf = self._pinned[slot].get(name)
        if buf is None or buf.numel() < n:
            size = max(n, 2 * buf.numel() if buf is not None else 0, 1)
            buf = self.torch.empty(size, dtype=dtype, pin_memory=True)
            self._pinned[slot][name] = buf
        return buf[:n].view(*shape)

    @property
    def slots(self):
        return len(self.streams)

    def prepare(self, req):
        """Host work: validate and build the plan.  Returns (plan, footprint)."""
        from .api import Plan
        if req.pos.ndim != 2 or req.pos.shape[1] != 3:
            raise ValueError("pos must be [N, 3]")
        if req.q.ndim != 2 or req.q.shape != (len(req.ps), req.pos.shape[0]):
            raise ValueError("q must be [C, N] with C = len(ps)")
        plan = Plan(req.box, req.ps, r_c=self.r_c, c=self.c, tol=self.tol, support=self.support,
                    max_atoms=max(1, req.n_atoms))
        N, C = req.n_atoms, len(req.ps)
        foot = plan.workspace_bytes + N * 12 * 2 + C * N * 4 + (3 * C + 1) * 8 + 48
        return plan, foot

    def launch(self, req, plan, slot):
        torch = self.torch
        st = self.streams[slot]
        N, C = req.n_atoms, len(req.ps)
        with torch.cuda.stream(st):
            pos_h = self._stage(slot, "pos", (N, 3), torch.float32)
            q_h = self._stage(slot, "q", (C, N), torch.float32)
            pos_h.copy_(torch.from_numpy(req.pos))
            q_h.copy_(torch.from_numpy(req.q))
            pos = pos_h.to(self.device, non_blocking=True)
            q = q_h.to(self.device, non_blocking=True)
            out = plan.execute(pos, q, forces=True, virial=True, stream=st)
            e_h = self._stage(slot, "energy", (3 * C + 1,), torch.float64)
            f_h = self._stage(slot, "forces", (N, 3), torch.float32)
            w_h = self._stage(slot, "virial", (6,), torch.float64)
            e_h.copy_(out["energy"], non_blocking=True)
            f_h.copy_(out["forces"], non_blocking=True)
            w_h.copy_(out["virial"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        # keep device tensors alive until the event completes
        return {"event": ev, "host": (e_h, f_h, w_h), "dev": (pos, q, out)}

    def done(self, token):
        return token["event"].query()

    def finish(self, req, token):
        e_h, f_h, w_h = token["host"]
        req.energy = e_h.numpy().copy()
        req.forces = f_h.numpy().copy()
        req.virial = w_h.numpy().copy()

    def budget_default(self):
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return int(0.5 * free)


class Server:
    """FIFO continuous batching with admission by HBM footprint.

    budget: bytes of device memory the in-flight requests may hold together.
    A request whose footprint alone exceeds the budget is rejected.
    """

    def __init__(self, executor, budget=None, plan_workers=0, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget) if budget is not None else executor.budget_default()
        self.pool = (concurrent.futures.ThreadPoolExecutor(max_workers=plan_workers)
                     if plan_workers > 0 else None)
        self.clock = clock
        self.pending = collections.deque()        # (req, future of (plan, footprint))
        self.inflight = {}                         # slot -> (req, plan, token)
        self.used = 0
        self.done = []
        self.peak_used = 0
        self.max_concurrency = 0
        self.t0 = None

    def now(self):
        return self.clock() - self.t0

    def submit(self, req):
        if self.t0 is None:
            self.t0 = self.clock()
        if self.pool is not None:
            fut = self.pool.submit(self.ex.prepare, req)
        else:
            fut = concurrent.futures.Future()
            try:
                fut.set_result(self.ex.prepare(req))
            except Exception as exc:  # failed at admission, reported there
                fut.set_exception(exc)
        self.pending.append((req, fut))

    def _retire(self):
        for slot in list(self.inflight):
            req, plan, token = self.inflight[slot]
            if self.ex.done(token):
                self.ex.finish(req, token)
                req.t_done = self.now()
                self.used -= req.footprint
                del self.inflight[slot]
                self.done.append(req)

    def _admit(self):
        free_slots = [s for s in range(self.ex.slots) if s not in self.inflight]
        while self.pending and free_slots:
            req, fut = self.pending[0]
            if not fut.done():
                break                               # FIFO: wait for the head's plan
            try:
                plan, foot = fut.result()
            except Exception as exc:                # malformed request: fail it, keep serving
                self.pending.popleft()
                req.error = "%s: %s" % (type(exc).__name__, exc)
                req.t_done = self.now()
                self.done.append(req)
                continue
            req.footprint = int(foot)
            if req.t_ready is None:
                req.t_ready = self.now()
            if foot > self.budget:
                self.pending.popleft()
                req.error = "footprint %d B exceeds the HBM budget %d B" % (foot, self.budget)
                req.t_done = self.now()
                self.done.append(req)
                continue
            if self.used + foot > self.budget:
                break                               # wait for memory to free up
            self.pending.popleft()
            slot = free_slots.pop(0)
            req.t_admit = self.now()
            self.used += foot
            self.peak_used = max(self.peak_used, self.used)
            self.inflight[slot] = (req, plan, self.ex.launch(req, plan, slot))
            self.max_concurrency = max(self.max_concurrency, len(self.inflight))

    def poll(self):
        self._retire()
        self._admit()

    def busy(self):
        return bool(self.pending or self.inflight)

    def run_trace(self, reqs, realtime=True, poll_sleep=50e-6):
        """Replay requests at their t_arrival offsets; return them when all
        have completed."""
        order = sorted(reqs, key=lambda r: r.t_arrival)
        # the cyclic garbage collector can pause the loop for tens of ms in
        # the middle of a trace; it runs before and after instead
        gc_on = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            self.t0 = self.clock()
            i = 0
            while i < len(order) or self.busy():
                now = self.now()
                while i < len(order) and (not realtime or order[i].t_arrival <= now):
                    if not realtime:
                        order[i].t_arrival = now
                    self.submit(order[i])
                    i += 1
                self.poll()
                if poll_sleep:
                    time.sleep(poll_sleep)
        finally:
            if gc_on:
                gc.enable()
        return order

    def close(self):
        if self.pool is not None:
            self.pool.shutdown(wait=True)


def latency_stats(reqs):
    lat = np.array([r.latency for r in reqs if r.error is None and r.latency is not None])
    if lat.size == 0:
        return {"n": 0}
    span = max(r.t_done for r in reqs if r.t_done is not None) - min(r.t_arrival for r in reqs)
    atoms = sum(r.n_atoms for r in reqs if r.error is None)
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_req_s": float(lat.size / span), "throughput_atoms_s": float(atoms / span)}


def make_requests(stream, ps=(1, 6), density=0.1):
    """Materialise a workloads.serving_stream trace as Requests."""
    from . import workloads as wl
    out = []
    for i, item in enumerate(stream):
        w = wl.random_box(item["n"], ps=ps, seed=item["seed"], density=density)
        out.append(Request(rid=i, pos=w["pos"], q=w["q"], box=tuple(w["box"]), ps=tuple(ps),
                           t_arrival=item["t"]))
    return out
