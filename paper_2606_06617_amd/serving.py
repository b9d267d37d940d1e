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
interval, so the pool only pays when plan building is slow.  The requests
admitted together in one poll (up to the executor's max_batch) run as one
batched launch on one slot.  Each request's result does not depend on what
else is in flight or what it was batched with: every kernel works on one
structure's own buffers and all reductions have a fixed order.

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
    """Runs requests through the C ABI on per-slot HIP streams.

    Every slot owns its device buffers (workspace, inputs, outputs) and its
    pinned host staging; both grow geometrically and are reused, so serving
    allocates nothing per request once the buffers have reached the sizes
    the trace needs (reserve() sizes them up front).  Several requests
    admitted together run as one pswflr_execute_batch call on one slot
    (one launch per stage for all of them)."""

    def __init__(self, slots=4, r_c=5.0, c=0.0, tol=1e-5, support=8, device="cuda:0", max_batch=16):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.r_c, self.c, self.tol, self.support = r_c, c, tol, support
        self.max_batch = int(max_batch)
        self._pinned = [dict() for _ in range(slots)]
        self._dev = [dict() for _ in range(slots)]

    def reserve(self, n_atoms, n_channels, workspace_bytes=0, n_requests=1):
        """Size every slot's pinned staging and device buffers for launches
        of up to n_requests requests holding n_atoms atoms and n_channels
        channels each, and a workspace of workspace_bytes, ahead of serving."""
        torch = self.torch
        na, nr = n_atoms * n_requests, n_requests
        for slot in range(self.slots):
            for store, pin in ((self._pinned[slot], True), (self._dev[slot], False)):
                self._buf(store, slot, "pos", 3 * na, torch.float32, pin)
                self._buf(store, slot, "q", n_channels * na, torch.float32, pin)
                self._buf(store, slot, "energy", (3 * n_channels + 1) * nr, torch.float64, pin)
                self._buf(store, slot, "forces", 3 * na, torch.float32, pin)
                self._buf(store, slot, "virial", 6 * nr, torch.float64, pin)
            if workspace_bytes:
                self._buf(self._dev[slot], slot, "ws", workspace_bytes * nr + (1 << 20), torch.uint8, False)
        torch.cuda.synchronize(self.device)

    def _buf(self, store, slot, name, n, dtype, pinned):
        buf = store.get(name)
        if buf is None or buf.numel() < n:
            size = max(n, 2 * buf.numel() if buf is not None else 0, 1)
            if pinned:
                buf = self.torch.empty(size, dtype=dtype, pin_memory=True)
            else:
                with self.torch.cuda.stream(self.streams[slot]):
                    buf = self.torch.empty(size, dtype=dtype, device=self.device)
            store[name] = buf
        return buf[:n]

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
        return self.launch_many([req], [plan], slot)

    def launch_many(self, reqs, plans, slot):
        """Stage the requests' inputs, run them (one execute, or one batched
        execute for several) on the slot's stream and queue the copies back."""
        import ctypes

        from . import _lib
        torch = self.torch
        st = self.streams[slot]
        pin, dev = self._pinned[slot], self._dev[slot]
        Ns = [r.n_atoms for r in reqs]
        Cs = [len(r.ps) for r in reqs]
        nq = sum(c * n for c, n in zip(Cs, Ns))
        ne = sum(3 * c + 1 for c in Cs)
        na = sum(Ns)
        n = len(reqs)
        pos_h = self._buf(pin, slot, "pos", 3 * na, torch.float32, True)
        q_h = self._buf(pin, slot, "q", nq, torch.float32, True)
        e_h = self._buf(pin, slot, "energy", ne, torch.float64, True)
        f_h = self._buf(pin, slot, "forces", 3 * na, torch.float32, True)
        w_h = self._buf(pin, slot, "virial", 6 * n, torch.float64, True)
        pos_d = self._buf(dev, slot, "pos", 3 * na, torch.float32, False)
        q_d = self._buf(dev, slot, "q", nq, torch.float32, False)
        e_d = self._buf(dev, slot, "energy", ne, torch.float64, False)
        f_d = self._buf(dev, slot, "forces", 3 * na, torch.float32, False)
        w_d = self._buf(dev, slot, "virial", 6 * n, torch.float64, False)
        pn, qn = pos_h.numpy(), q_h.numpy()
        a0 = q0 = 0
        for r, N, C in zip(reqs, Ns, Cs):
            pn[3 * a0:3 * (a0 + N)] = r.pos.reshape(-1)
            qn[q0:q0 + C * N] = r.q.reshape(-1)
            a0 += N
            q0 += C * N
        L = _lib.lib()
        with torch.cuda.stream(st):
            pos_d.copy_(pos_h, non_blocking=True)
            q_d.copy_(q_h, non_blocking=True)
            sptr = ctypes.c_void_p(st.cuda_stream)
            if n == 1:
                ws = self._buf(dev, slot, "ws", plans[0].workspace_bytes, torch.uint8, False)
                _lib.check(L.pswflr_execute(plans[0].handle, sptr, ws.data_ptr(), ws.numel(), Ns[0],
                                            pos_d.data_ptr(), q_d.data_ptr(), e_d.data_ptr(), f_d.data_ptr(),
                                            w_d.data_ptr(), None))
            else:
                handles = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
                natoms = (ctypes.c_int64 * n)(*Ns)
                need = ctypes.c_size_t()
                _lib.check(L.pswflr_batch_workspace(n, handles, natoms, ctypes.byref(need)))
                ws = self._buf(dev, slot, "ws", need.value, torch.uint8, False)
                ios = (_lib.IO * n)()
                pb, qb, eb, fb, wb = (pos_d.data_ptr(), q_d.data_ptr(), e_d.data_ptr(), f_d.data_ptr(),
                                      w_d.data_ptr())
                a0 = q0 = e0 = 0
                for i, (N, C) in enumerate(zip(Ns, Cs)):
                    io = ios[i]
                    io.n_atoms = N
                    io.pos = pb + 12 * a0
                    io.q = qb + 4 * q0
                    io.energy = eb + 8 * e0
                    io.forces = fb + 12 * a0
                    io.virial = wb + 48 * i
                    io.potential = None
                    a0 += N
                    q0 += C * N
                    e0 += 3 * C + 1
                _lib.check(L.pswflr_execute_batch(n, handles, ios, sptr, ws.data_ptr(), ws.numel()))
            e_h.copy_(e_d, non_blocking=True)
            f_h.copy_(f_d, non_blocking=True)
            w_h.copy_(w_d, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"event": ev, "host": (e_h, f_h, w_h), "sizes": (Ns, Cs), "plans": plans}

    def done(self, token):
        return token["event"].query()

    def finish_many(self, reqs, token):
        e_h, f_h, w_h = token["host"]
        en, fn, wn = e_h.numpy(), f_h.numpy(), w_h.numpy()
        Ns, Cs = token["sizes"]
        a0 = e0 = 0
        for i, (r, N, C) in enumerate(zip(reqs, Ns, Cs)):
            r.energy = en[e0:e0 + 3 * C + 1].copy()
            r.forces = fn[3 * a0:3 * (a0 + N)].reshape(N, 3).copy()
            r.virial = wn[6 * i:6 * i + 6].copy()
            a0 += N
            e0 += 3 * C + 1

    def finish(self, req, token):
        self.finish_many([req], token)

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
        self.inflight = {}                         # slot -> (requests, token)
        self.used = 0
        self.done = []
        self.peak_used = 0
        self.max_concurrency = 0                   # launches in flight at once
        self.max_inflight_requests = 0             # requests in flight at once
        self.max_coalesced = 0
        self.launches = 0
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
            reqs, token = self.inflight[slot]
            if self.ex.done(token):
                if len(reqs) == 1:
                    self.ex.finish(reqs[0], token)
                else:
                    self.ex.finish_many(reqs, token)
                t = self.now()
                for req in reqs:
                    req.t_done = t
                    self.used -= req.footprint
                    self.done.append(req)
                del self.inflight[slot]

    def _admit(self):
        """Admit head-of-queue requests in FIFO order while a slot is free and
        their footprints fit the budget; the requests admitted for one slot
        in one poll (up to the executor's max_batch) run as one launch."""
        max_batch = getattr(self.ex, "max_batch", 1)
        free_slots = [s for s in range(self.ex.slots) if s not in self.inflight]
        while self.pending and free_slots:
            group, plans = [], []
            while self.pending and len(group) < max_batch:
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
                req.t_admit = self.now()
                self.used += foot
                group.append(req)
                plans.append(plan)
            if not group:
                break
            self.peak_used = max(self.peak_used, self.used)
            slot = free_slots.pop(0)
            if len(group) == 1:
                token = self.ex.launch(group[0], plans[0], slot)
            else:
                token = self.ex.launch_many(group, plans, slot)
            self.inflight[slot] = (group, token)
            self.launches += 1
            self.max_concurrency = max(self.max_concurrency, len(self.inflight))
            self.max_inflight_requests = max(self.max_inflight_requests,
                                             sum(len(g) for g, _ in self.inflight.values()))
            self.max_coalesced = max(self.max_coalesced, len(group))

    def poll(self):
        self._retire()
        self._admit()

    def busy(self):
        return bool(self.pending or self.inflight)

    def run_trace(self, reqs, realtime=True, poll_sleep=50e-6):
        """Replay requests at their t_arrival offsets; return them when all
        have completed.  While work is on the device the loop polls without
        sleeping (a sleep adds its own length to every completion it
        overlaps); with nothing in flight it sleeps until the next arrival,
        at most poll_sleep seconds at a time."""
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
                if poll_sleep and not self.inflight and not self.pending:
                    wait = poll_sleep
                    if realtime and i < len(order):
                        wait = min(wait, order[i].t_arrival - self.now())
                    if wait > 0:
                        time.sleep(wait)
        finally:
            if gc_on:
                gc.enable()
        return order

    def close(self):
        if self.pool is not None:
            self.pool.shutdown(wait=True)


def latency_stats(reqs):
    """Latency percentiles (arrival to completion) and the phases behind
    them: ready (plan built) - arrival, admit - ready (waiting for a slot or
    memory), done - admit (device work and copies)."""
    ok = [r for r in reqs if r.error is None and r.latency is not None]
    if not ok:
        return {"n": 0}
    lat = np.array([r.latency for r in ok])
    span = max(r.t_done for r in reqs if r.t_done is not None) - min(r.t_arrival for r in reqs)
    atoms = sum(r.n_atoms for r in ok)
    plan = np.array([r.t_ready - r.t_arrival for r in ok])
    wait = np.array([r.t_admit - r.t_ready for r in ok])
    serv = np.array([r.t_done - r.t_admit for r in ok])
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3),
            "throughput_req_s": float(lat.size / span), "throughput_atoms_s": float(atoms / span),
            "plan_p99_ms": float(np.percentile(plan, 99) * 1e3), "plan_max_ms": float(plan.max() * 1e3),
            "wait_p99_ms": float(np.percentile(wait, 99) * 1e3), "wait_max_ms": float(wait.max() * 1e3),
            "service_p99_ms": float(np.percentile(serv, 99) * 1e3), "service_max_ms": float(serv.max() * 1e3)}


def make_requests(stream, ps=(1, 6), density=0.1):
    """Materialise a workloads.serving_stream trace as Requests."""
    from . import workloads as wl
    out = []
    for i, item in enumerate(stream):
        w = wl.random_box(item["n"], ps=ps, seed=item["seed"], density=density)
        out.append(Request(rid=i, pos=w["pos"], q=w["q"], box=tuple(w["box"]), ps=tuple(ps),
                           t_arrival=item["t"]))
    return out
