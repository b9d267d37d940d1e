"""Throughput benchmark of the PSWF-LR reciprocal-space path on one MI355X.

A step is one whole evaluation (sort, spread, forward FFT with the fused
kernel scaling and energy/virial reduction, inverse FFT, gather of forces)
of the default workload, the 1e6-atom ionic frame (12 channels, 256^3
grid, P = 8), with inputs resident in HBM.  Prints one JSON line with the
throughput (atoms/s), the roofline fraction of the dominant kernel from
HIP events recorded around every launch during the timed steps, and the
FP64 oracle timed on a bounded sample of the same workload on the host.

  python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload ionic_1m]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LR energy+force atoms/s at ≤1e-4 rel force err; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32, published
STAGES = ["sort", "qsum", "spread", "fft_z", "fft_y", "fft_x_scale", "reduce", "ifft_y", "ifft_z", "gather"]
C_MOL, R_C = 12.024, 5.0


def workload(name):
    from paper_2606_06617_amd import workloads as wl
    if name == "ionic_1m":
        return wl.ionic()
    if name == "water_3000":
        return wl.water()
    if name == "nacl_512":
        return wl.nacl()
    raise SystemExit("unknown workload %s" % name)


def algorithmic_bytes(info, N, C, cg_spread):
    """HBM bytes each kernel must move per launch (reads + writes of the
    data it consumes and produces once), the roofline numerator."""
    Mx, My, Mz = info["grid"]
    M = Mx * My * Mz
    KZ, NY, xcols = info["kz_keep"], info["ny_keep"], info["xcols"]
    s1 = 8 * C * Mx * My * KZ
    s2 = 8 * C * Mx * NY * KZ
    return {
        "spread": 16 * N + 4 * cg_spread * N + 4 * cg_spread * M,
        "fft_z": 4 * C * M + s1,
        "fft_y": s1 + s2,
        "fft_x_scale": 2 * 8 * C * Mx * xcols,
        "ifft_y": 8 * C * Mx * xcols + s1,
        "ifft_z": s1 + 4 * C * M,
        "gather": 4 * C * M + N * (16 + 4 * C) + 12 * N,
    }


def algorithmic_flops(info, N, C):
    """FP32 operations the method needs per launch where they, not bytes,
    bound a kernel: spreading 2 P^3 N C (one FMA per window point and
    channel), gathering 8 P^3 N C (potential and gradient sums)."""
    P = info["support"]
    return {"spread": 2 * P ** 3 * N * C, "gather": 8 * P ** 3 * N * C}


def stage_kernel(stage, info):
    """Name (as in rocprofv3 summaries) of the kernel a timed stage launches;
    the spread is instantiated per support, z blocks per tile edge and
    channel accumulators."""
    P = info["support"]
    nbz = (info["tile"][2] + 3) // 4
    cg = int(info["cg_spread"])
    cgt = 2 if cg <= 2 else (4 if cg <= 4 else 12)   # accumulator counts the spread is built for
    return {"spread": "k_spread<%d,%d,%d>" % (P, nbz, cgt), "fft_z": "k_zfwd", "fft_y": "k_yfwd", "fft_x_scale": "k_xmul",
            "ifft_y": "k_yinv", "ifft_z": "k_zinv", "gather": "k_gather<%d>" % P}.get(stage)


def measured_traffic(workload_name, kernel):
    """HBM bytes per dispatch of `kernel` from the committed counter summary
    of this workload, or None when there is none or the kernel source has
    changed since the counters were taken."""
    from paper_2606_06617_amd import profiling
    rows, sha = profiling.read_traffic(os.path.join(ROOT, "profiles", "traffic_%s.txt" % workload_name))
    if not rows or sha != profiling.source_hash():
        return None
    if kernel in rows:
        return rows[kernel]
    # kernels instantiated on a path flag (k_zfwd<true> for k_zfwd): the one launched
    hits = [v for k, v in rows.items() if k.startswith(kernel + "<")]
    return hits[0] if len(hits) == 1 else None


def batch_leg(reps=10):
    """The 64-structure training batch (N in [200, 4000], grids 24^3-64^3,
    p = 1 and 6): one batched call on flat arrays (a launch per stage over
    all structures) with forces and virial, against the same structures
    evaluated one call after another, both with workspaces and outputs
    reused; and the training step of the batch: energy-only batched forward
    plus the batched hand-written adjoint (dE/dq, dE/dr of every structure).
    The plans take the planner's tiles; the batched call is timed again with
    the tiles the autotuner picks one structure at a time.  atoms/s over the
    batch, host wall time per call."""
    import torch

    from paper_2606_06617_amd import workloads as wl
    from paper_2606_06617_amd.api import Batch, Plan

    structs = wl.diff_batch()
    dev = torch.device("cuda:0")
    plans = [Plan(st["box"], st["ps"], r_c=R_C, c=C_MOL, grid=st["grid"], support=st["support"] or 0,
                  max_atoms=st["pos"].shape[0], autotune=False) for st in structs]
    inputs = [(torch.from_numpy(st["pos"]).to(dev), torch.from_numpy(st["q"]).to(dev)) for st in structs]
    batch = Batch(plans, [x[0].shape[0] for x in inputs])
    pos, q = Batch.concat(inputs)
    atoms = batch.atoms
    ws = batch.new_workspace(dev)
    out = batch.execute(pos, q, forces=True, virial=True, workspace=ws)
    for _ in range(2):
        batch.execute(pos, q, forces=True, virial=True, workspace=ws, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.execute(pos, q, forces=True, virial=True, workspace=ws, out=out)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    g = torch.ones(sum(batch.Cs), dtype=torch.float64, device=dev)
    eo = {"energy": torch.empty(batch.elen, dtype=torch.float64, device=dev)}
    for _ in range(2):
        batch.execute(pos, q, forces=False, virial=False, workspace=ws, out=eo)
        batch.backward(ws, pos, q, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.execute(pos, q, forces=False, virial=False, workspace=ws, out=eo)
        batch.backward(ws, pos, q, g)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / reps
    wss = [p.new_workspace(dev) for p in plans]
    for p, (ps_, qs_), w_ in zip(plans, inputs, wss):
        p.execute(ps_, qs_, forces=True, virial=True, workspace=w_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for p, (ps_, qs_), w_ in zip(plans, inputs, wss):
            p.execute(ps_, qs_, forces=True, virial=True, workspace=w_)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    t_tuned = _batch_with_tuned_tiles(structs, inputs, plans, reps)
    return {"structures": len(structs), "atoms": atoms, "support": plans[0].info["support"],
            "batched_ms": round(t_batch * 1e3, 3), "batched_atoms_s": round(atoms / t_batch, 1),
            "batched_standalone_tuned_tiles_ms": round(t_tuned * 1e3, 3),
            "forward_adjoint_ms": round(t_train * 1e3, 3), "forward_adjoint_atoms_s": round(atoms / t_train, 1),
            "sequential_ms": round(t_seq * 1e3, 3), "sequential_atoms_s": round(atoms / t_seq, 1)}


def _batch_with_tuned_tiles(structs, inputs, plans, reps):
    """The same batched call with each structure's tile from the autotuner
    (timed one structure at a time, cached in a temporary file): host wall
    time per call."""
    import tempfile

    import torch

    from paper_2606_06617_amd import autotune
    from paper_2606_06617_amd.api import Batch, Plan

    old = os.environ.get("PSWFLR_AUTOTUNE_CACHE")
    with tempfile.TemporaryDirectory() as tdir:
        os.environ["PSWFLR_AUTOTUNE_CACHE"] = os.path.join(tdir, "tune.json")
        try:
            best, tuned = {}, []
            for st, (pos, q), p in zip(structs, inputs, plans):
                key = (p.info["grid"], p.info["support"], p.C, autotune.key_for("", p.info["grid"], p.info["support"],
                                                                               p.C, pos.shape[0]))
                if key not in best:
                    best[key] = autotune.tune(pos, q, st["box"], st["ps"], r_c=R_C, c=C_MOL, grid=p.info["grid"],
                                              support=p.info["support"], reps=10)
                tuned.append(Plan(st["box"], st["ps"], r_c=R_C, c=C_MOL, grid=p.info["grid"],
                                  support=p.info["support"], max_atoms=pos.shape[0], tile=best[key]))
        finally:
            if old is None:
                os.environ.pop("PSWFLR_AUTOTUNE_CACHE", None)
            else:
                os.environ["PSWFLR_AUTOTUNE_CACHE"] = old
    dev = inputs[0][0].device
    batch = Batch(tuned, [x[0].shape[0] for x in inputs])
    pos, q = Batch.concat(inputs)
    ws = batch.new_workspace(dev)
    out = batch.execute(pos, q, forces=True, virial=True, workspace=ws)
    for _ in range(2):
        batch.execute(pos, q, forces=True, virial=True, workspace=ws, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.execute(pos, q, forces=True, virial=True, workspace=ws, out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _call_latency(plan, pos, q, reps):
    """Host wall time of one call plus a stream synchronisation (eager), of a
    replay of the call captured once as a HIP graph, and the device time of
    the call's kernels (HIP events around every launch)."""
    import ctypes

    import torch

    from paper_2606_06617_amd import _lib

    L = _lib.lib()
    dev = pos.device
    N, C = pos.shape[0], plan.C
    ws = plan.new_workspace(dev)
    res = {"energy": torch.empty(3 * C + 1, dtype=torch.float64, device=dev),
           "forces": torch.empty((N, 3), dtype=torch.float32, device=dev),
           "virial": torch.empty(6, dtype=torch.float64, device=dev)}
    side = torch.cuda.Stream(device=dev)

    def call():
        plan.execute(pos, q, forces=True, virial=True, workspace=ws, out=res, stream=side)

    with torch.cuda.stream(side):
        for _ in range(10):
            call()
    side.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
        side.synchronize()
    eager = (time.perf_counter() - t0) / reps
    ref = res["energy"].clone()
    graph_ms = None
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            call()
        side.synchronize()
        for _ in range(10):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
            torch.cuda.synchronize()
        graph_ms = round((time.perf_counter() - t0) / reps * 1e3, 4)
        if not torch.equal(res["energy"], ref):
            graph_ms = None
    except RuntimeError:
        graph_ms = None
    _lib.check(L.pswflr_profile_enable(plan.handle, 1))
    with torch.cuda.stream(side):
        for _ in range(20):
            call()
    side.synchronize()
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int64 * len(STAGES))()
    _lib.check(L.pswflr_profile_read(plan.handle, ms, cnt))
    _lib.check(L.pswflr_profile_enable(plan.handle, 0))
    return {"tile": list(plan.info["tile"]), "eager_call_ms": round(eager * 1e3, 4), "graph_replay_ms": graph_ms,
            "device_ms": round(sum(ms) / 20, 4), "launches_per_call": int(sum(cnt) // 20)}


def small_leg(reps=200):
    """Per-call latency of the two small configurations (rock-salt 512 atoms
    at 32^3, P = 6; water 3000 atoms, two channels, at 48^3, P = 8), energy,
    forces and virial: launch-bound work of a few microseconds per kernel.
    Each is timed with the planner's tile and again with the tile the
    autotuner picks for it (timed candidates, cached in a temporary file)."""
    import tempfile

    import torch

    from paper_2606_06617_amd import autotune
    from paper_2606_06617_amd import workloads as wl
    from paper_2606_06617_amd.api import Plan

    out = {}
    old = os.environ.get("PSWFLR_AUTOTUNE_CACHE")
    with tempfile.TemporaryDirectory() as tdir:
        os.environ["PSWFLR_AUTOTUNE_CACHE"] = os.path.join(tdir, "tune.json")
        try:
            for w in (wl.nacl(), wl.water()):
                N, C = w["pos"].shape[0], len(w["ps"])
                dev = torch.device("cuda:0")
                pos = torch.from_numpy(w["pos"]).to(dev)
                q = torch.from_numpy(w["q"]).to(dev)
                plan = Plan(w["box"], w["ps"], r_c=R_C, c=C_MOL, grid=w["grid"], support=w["support"],
                            max_atoms=N)
                rec = {"grid": list(plan.info["grid"]), "support": plan.info["support"], "channels": C}
                rec.update(_call_latency(plan, pos, q, reps))
                best = autotune.tune(pos, q, w["box"], w["ps"], r_c=R_C, c=C_MOL, grid=w["grid"],
                                     support=w["support"], reps=20)
                tuned = Plan(w["box"], w["ps"], r_c=R_C, c=C_MOL, grid=w["grid"], support=w["support"],
                             max_atoms=N, tile=best)
                rec["autotuned"] = _call_latency(tuned, pos, q, reps)
                out[w["name"]] = rec
        finally:
            if old is None:
                os.environ.pop("PSWFLR_AUTOTUNE_CACHE", None)
            else:
                os.environ["PSWFLR_AUTOTUNE_CACHE"] = old
    return out


def serving_leg(nreq=2000, seed=6, fractions=(0.5, 0.8, 0.95), slots=4, max_batch=16):
    """Continuous-batching latency on the Poisson request mix (sizes
    log-uniform in [100, 5e4] atoms, density 0.1, channels p = 1 and 6,
    tolerance 1e-5): the one-at-a-time capacity is measured first (one
    slot, one request per launch, back to back), then the same requests
    arrive as Poisson processes at the given fractions of it and are served
    with `slots` overlapping launches, the requests admitted together
    coalesced into one batched launch (up to max_batch).  Latency =
    completion - arrival, including the host plan, both copies and the
    evaluation; the phases behind the tail (plan, wait for a slot, service)
    are reported with it.  Every buffer is sized before the timed traces and
    a warm-up trace runs on the executor the rates use."""
    from paper_2606_06617_amd import workloads as wl
    from paper_2606_06617_amd.serving import HipExecutor, Server, latency_stats, make_requests

    stream = wl.serving_stream(nreq=nreq, rate=1.0, seed=seed)
    reqs = make_requests(stream)
    # warm the host caches that plans of any box share (window bandwidth
    # grid, kernel fits), and size the buffers for the largest request
    ex1 = HipExecutor(slots=1, max_batch=1)
    max_ws = max(ex1.prepare(r)[0].workspace_bytes for r in reqs)
    maxn, maxc = max(r.n_atoms for r in reqs), max(len(r.ps) for r in reqs)
    ex1.reserve(maxn, maxc, max_ws)
    warm = Server(ex1)
    warm.run_trace(reqs[:32], realtime=False)
    solo = Server(ex1)
    t0 = time.perf_counter()
    solo.run_trace(reqs, realtime=False)
    span = time.perf_counter() - t0
    capacity = nreq / span
    atoms = sum(r.n_atoms for r in reqs)
    out = {"requests_per_rate": nreq, "capacity_req_s": round(capacity, 1),
           "capacity_atoms_s": round(atoms / span, 1), "atoms_per_request": "log-uniform [100, 50000]",
           "slots": slots, "max_batch": max_batch, "rates": []}
    ex = HipExecutor(slots=slots, max_batch=max_batch)
    ex.reserve(maxn, maxc, max_ws, n_requests=max_batch)
    rng = np.random.default_rng(seed + 1)

    def replay(f, subset):
        gaps = rng.exponential(1.0 / (f * capacity), size=len(subset))
        for r, t in zip(subset, np.cumsum(gaps)):
            r.t_arrival, r.t_done, r.t_admit, r.t_ready, r.error = float(t), None, None, None, None
        srv = Server(ex)
        res = srv.run_trace(subset, realtime=True)
        srv.close()
        return srv, res

    # untimed warm-up: the whole trace at the first rate on the executor the
    # rates use.  The first full trace on a fresh executor has shown one
    # stall of about 8 ms (one launch's device work, with the plan built
    # behind it waiting), never seen in a repeat of the same trace.
    replay(fractions[0], reqs)
    for f in fractions:
        srv, res = replay(f, reqs)
        st = latency_stats(res)
        out["rates"].append({"load": f, "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                             "mean_ms": round(st["mean_ms"], 3), "max_ms": round(st["max_ms"], 3),
                             "req_s": round(st["throughput_req_s"], 1),
                             "atoms_s": round(st["throughput_atoms_s"], 1),
                             "wait_p99_ms": round(st["wait_p99_ms"], 3), "wait_max_ms": round(st["wait_max_ms"], 3),
                             "service_p99_ms": round(st["service_p99_ms"], 3),
                             "service_max_ms": round(st["service_max_ms"], 3),
                             "plan_p99_ms": round(st["plan_p99_ms"], 3),
                             "max_concurrency": srv.max_concurrency,
                             "max_inflight_requests": srv.max_inflight_requests, "launches": srv.launches,
                             "max_coalesced": srv.max_coalesced})
    return out


def _oracle_channel_timing(args):
    """One worker of the CPU baseline: the FP64 direct sum (E, F, W) of one
    channel on 0 and on n atoms, single-threaded; returns both times."""
    pos, q, box, p = args
    from threadpoolctl import threadpool_limits

    from oracle import reciprocal
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        reciprocal.evaluate(pos[:0], q[:, :0], box, [p], C_MOL, R_C)
        t1 = time.perf_counter()
        reciprocal.evaluate(pos, q, box, [p], C_MOL, R_C)
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def cpu_baseline(w, n_sample=128):
    """The FP64 oracle (the direct structure-factor sum over the k-ball with
    energy, forces and virial) timed on the host's cores: channels are
    independent evaluations, so one worker process per channel (up to the
    cores this process may run on, os.sched_getaffinity), each timing its
    channel with no atoms (the fixed cost of the k-ball) and with the first
    n_sample atoms.  The oracle's cost is linear in atoms, so a channel of
    the full frame takes t_0 + N (t_n - t_0) / n; the frame takes the
    slowest worker's channel time for every round of workers the channels
    need, and value = N / that."""
    import multiprocessing as mp

    N, C = w["pos"].shape[0], len(w["ps"])
    ncores = len(os.sched_getaffinity(0))
    workers = max(1, min(C, ncores))
    pos = np.ascontiguousarray(w["pos"][:n_sample].astype(np.float64))
    tasks = [(pos, w["q"][c:c + 1, :n_sample].astype(np.float64), np.asarray(w["box"]), w["ps"][c])
             for c in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        times = pool.map(_oracle_channel_timing, tasks)
    per_chan = max(t0 + N * (tn - t0) / n_sample for t0, tn in times)
    rounds = -(-C // workers)
    full = rounds * per_chan
    return {"value": N / full, "unit": "atoms/s", "cores": workers, "kind": "oracle",
            "sample": ("FP64 direct sum over the k-ball |k|<=c/r_c, E+F+W, one single-threaded worker per channel "
                       "(%d workers on %d available cores, channels %d..%d, p=%s), each timed on 0 and the first %d "
                       "atoms (t_0 %.2f-%.2f s, t_n %.2f-%.2f s); extrapolated linearly to %d atoms: %.3g s per "
                       "channel, %d round(s) for %d channels = %.3g s"
                       % (workers, ncores, 0, workers - 1, sorted(set(w["ps"][:workers])), n_sample,
                          min(t[0] for t in times), max(t[0] for t in times), min(t[1] for t in times),
                          max(t[1] for t in times), N, per_chan, rounds, C, full))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ionic_1m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the continuous-batching latency leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-structure batch leg")
    ap.add_argument("--no-small", action="store_true", help="skip the small-configuration latency leg")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also launch one plain device-to-device copy of this many MiB (a known-size "
                         "kernel that calibrates FETCH_SIZE / WRITE_SIZE counter readings)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each structure, or each "
              "channel group of one structure, runs whole on one device); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import ctypes

    import torch

    from paper_2606_06617_amd import _lib
    from paper_2606_06617_amd.api import Plan

    w = workload(args.workload)
    N = w["pos"].shape[0]
    C = len(w["ps"])
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(w["pos"]).to(dev)
    q = torch.from_numpy(w["q"]).to(dev)
    plan = Plan(w["box"], w["ps"], r_c=R_C, c=C_MOL, grid=w["grid"], support=w["support"], max_atoms=N)
    ws = plan.new_workspace(dev)
    out = {"energy": torch.empty(3 * C + 1, dtype=torch.float64, device=dev),
           "forces": torch.empty((N, 3), dtype=torch.float32, device=dev),
           "virial": torch.empty(6, dtype=torch.float64, device=dev)}
    L = _lib.lib()

    def step():
        plan.execute(pos, q, forces=True, virial=True, workspace=ws, out=out)

    def profiled(mask, steps):
        # steps calls with the stages in mask bracketed by HIP events on the
        # call's stream: (wall ms per step, per-stage ms per step, per-stage
        # average launch ms)
        _lib.check(L.pswflr_profile_stages(plan.handle, mask))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _lib.check(L.pswflr_profile_read(plan.handle, ms, cnt))
        _lib.check(L.pswflr_profile_stages(plan.handle, 0))
        return ((t1 - t0) * 1e3 / steps, {STAGES[i]: ms[i] / steps for i in range(len(STAGES))},
                {STAGES[i]: (ms[i] / cnt[i] if cnt[i] else 0.0) for i in range(len(STAGES))})

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    info = plan.info
    cg_spread = int(info["cg_spread"])
    algo = algorithmic_bytes(info, N, C, cg_spread)
    flops = algorithmic_flops(info, N, C)
    # per-stage breakdown from an untimed pass with every stage bracketed
    # (the event records add about 0.05 ms per step); the timed steps then
    # bracket only the dominant kernel, whose launch time gives the roofline
    _, stage_ms, stage_launch_ms = profiled((1 << len(STAGES)) - 1, args.steps)
    dom = max(algo.keys(), key=lambda k: stage_ms[k])
    ms_per_step, timed_ms, timed_launch_ms = profiled(1 << STAGES.index(dom), args.steps)
    avg_launch_ms = dict(stage_launch_ms)
    avg_launch_ms[dom] = timed_launch_ms[dom]
    t_dom = avg_launch_ms[dom] * 1e-3
    traffic = measured_traffic(args.workload, stage_kernel(dom, info))
    if flops.get(dom, 0) / (FP32_PEAK_TFLOPS * 1e12) > algo[dom] / (HBM_PEAK_GBS * 1e9):
        achieved = flops[dom] / t_dom / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                    "traffic": None if traffic is None else int(traffic),
                    "algorithmic_flops_per_launch": int(flops[dom]), "avg_launch_ms": round(avg_launch_ms[dom], 4)}
    else:
        achieved = algo[dom] / t_dom / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else int(traffic),
                    "algorithmic_bytes_per_launch": int(algo[dom]), "avg_launch_ms": round(avg_launch_ms[dom], 4)}
    per_stage = {k: {"ms_per_step": round(stage_ms[k], 4),
                     "GB_s": (round(algo[k] / (avg_launch_ms[k] * 1e-3) / 1e9, 1)
                              if k in algo and avg_launch_ms[k] > 0 else None)} for k in STAGES}

    rec = {
        "metric": METRIC,
        "value": N / (ms_per_step * 1e-3),
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_atoms": N, "channels": C, "p": sorted(set(w["ps"])),
                   "grid": list(info["grid"]), "support": info["support"], "c": info["c"], "r_c": info["r_c"],
                   "c_spread": round(info["c_spread"], 4), "eta": round(info["eta"], 4),
                   "box": [round(b, 4) for b in w["box"]], "outputs": "energy+forces+virial"},
        "roofline": roofline,
        "stages": per_stage,
    }
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["calib_copy_bytes"] = 2 * src.numel() * 4
    if not args.no_batch:
        rec["batch"] = batch_leg()
    if not args.no_small:
        rec["small"] = small_leg()
    if not args.no_serving:
        rec["serving"] = serving_leg()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
