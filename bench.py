"""Benchmark: RPCA pixel-frames/s per ALM iteration on one MI355X.

Workload: the seeded 512x512-pixel x 20-frame ultrasound window (Casorati
262144 x 20), FP32, lambda = 1/512, tol = 1e-6, maxit = 1000.  One step is
one complete solve (init pass, every iteration, finalize) with the input
already resident in HBM, on the production path (graph-captured iteration
chunks).

value = sum over timed steps of m * n * iterations / wall time of the steps.

The JSON line also carries
  roofline     : the fused update kernel's algorithmic bytes per launch over
                 its mean launch time (a HIP start/stop event pair that each
                 launch records on its own stream from its dispatch packet,
                 over a repeat of the timed steps) against
                 the 8 TB/s HBM peak, and the HBM bytes per launch measured
                 with rocprofv3 counters (profiles/);
  cpu_baseline : the FP64 CPU oracle timed on a bounded number of iterations
                 of the same window on this host;
  latency      : p50 / p99 of the per-solve wall time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "RPCA pixel-frames/s per ALM iter; p50/p99 solve latency, 20-frame windows"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "update_traffic_512x512x20_f32.json")
KERNEL_SOURCES = ("paper_2506_10257_amd/csrc/stream_impl.h", "paper_2506_10257_amd/csrc/common.h",
                  "paper_2506_10257_amd/csrc/stream_f32.hip")


def tuning_summary() -> dict:
    """Current tuning choices (eigensolver threads per class; classes on the
    MFMA tile kernel)."""
    import paper_2506_10257_amd as rp
    ch = rp.tuning_choices()
    return {"eig_threads_f32": {str(c): v for (dt, c), v in ch["eig_threads"].items() if dt == rp.RPCA_F32},
            "eig_threads_f64": {str(c): v for (dt, c), v in ch["eig_threads"].items() if dt == rp.RPCA_F64},
            "tile_kernel_classes": [c for c, v in ch["stream_kernel"].items() if v == 1],
            "tile_rows": {str(nb): v for nb, v in ch["tile_rows"].items()},
            "reg_tiles_f32": {str(c): v for (dt, c), v in ch["reg_tiles"].items() if dt == rp.RPCA_F32},
            "reg_tiles_f64": {str(c): v for (dt, c), v in ch["reg_tiles"].items() if dt == rp.RPCA_F64}}


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per update launch from the committed rocprofv3 counter
    summary, or None when absent or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(X, lam, budget_s: float = 12.0, max_iters: int = 40, one_thread_iters: int = 3):
    """FP64 oracle on this host: iterations of the same window until the
    budget is used (tol = 0 runs a fixed count) with the BLAS pool as it is,
    then a few iterations with the pool limited to one thread."""
    import numpy as np
    from oracle import rpca
    threads, limits = None, None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        info = threadpool_info()
        threads = max((d.get("num_threads") or 0) for d in info) if info else None
        limits = threadpool_limits
    except Exception:
        pass
    m, n = X.shape
    X64 = np.asarray(X, dtype=np.float64)
    t0 = time.perf_counter()
    rpca(X64, lam=lam, tol=0.0, maxit=1)
    one = time.perf_counter() - t0
    iters = int(max(1, min(max_iters, budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    rpca(X64, lam=lam, tol=0.0, maxit=iters)
    dt = time.perf_counter() - t0
    out = {"value": m * n * iters / dt, "unit": "pixel-frames/s per ALM iter",
           "cores": threads or len(os.sched_getaffinity(0)), "kind": "oracle",
           "sample": f"{iters} FP64 ALM iterations (full SVD) of the {m}x{n} window, tol=0",
           "s_per_iter": dt / iters, "host_cpus": len(os.sched_getaffinity(0))}
    if limits is not None and one_thread_iters > 0:
        with limits(limits=1):
            t0 = time.perf_counter()
            rpca(X64, lam=lam, tol=0.0, maxit=one_thread_iters)
            d1 = time.perf_counter() - t0
        out["one_thread"] = {"value": m * n * one_thread_iters / d1, "iters": one_thread_iters,
                             "s_per_iter": d1 / one_thread_iters}
    return out


def _gen_batch_window(args):
    from synth import batch_window
    H, W, n, seed = args
    return batch_window(H, W, n, seed).X().astype("float32")


def batch_measure(count: int, steps: int, warmup: int) -> dict:
    """The 64-window batch (sizes {256^2, 384x512, 512^2, 512x768} x frames
    {10, 20, 40, 60}, FP32, tol 1e-6, maxit 1000) solved together by
    rpca_solve_many, against the plain path that solves the same windows one
    call at a time.  Returns the figures of the batched path (throughput,
    solves/s, per-iteration HBM fraction, kernel split) and of the plain path."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor

    import paper_2506_10257_amd as rp
    from synth import batch_shapes

    dev = torch.device("cuda:0")
    shapes = batch_shapes(count)
    workers = min(16, len(os.sched_getaffinity(0)))
    with ProcessPoolExecutor(workers) as ex:
        Xs = list(ex.map(_gen_batch_window, shapes))
    Ms = [torch.from_numpy(np.ascontiguousarray(X.T)).to(dev).t() for X in Xs]
    elems = [X.shape[0] * X.shape[1] for X in Xs]
    del Xs
    tol, maxit = 1e-6, 1000
    torch.cuda.synchronize()
    print(f"[batch] {len(Ms)} windows, {sum(elems) / 1e6:.0f} M elements", file=sys.stderr, flush=True)

    for _ in range(warmup):
        rp.solve_many(Ms, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    walls, work = [], 0
    for _ in range(steps):
        t0 = time.perf_counter()
        res = rp.solve_many(Ms, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        work += sum(e * r.iterations for e, r in zip(elems, res))
    wall = sum(walls)
    iters = [r.iterations for r in res]

    # One more step with kernel timing: the library then runs every solve on
    # one stream with direct launches, each recording a HIP start/stop event pair.
    rp.rpca_profile_read(reset=True)
    rp.rpca_profile_enable(True)
    t0 = time.perf_counter()
    rp.solve_many(Ms, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    timed_wall = time.perf_counter() - t0
    rp.rpca_profile_enable(False)
    prof = rp.rpca_profile_read(reset=True)
    print(f"[batch] batched: {len(Ms) * steps / wall:.2f} solves/s", file=sys.stderr, flush=True)

    # plain path: one solve per call, in order
    t0 = time.perf_counter()
    plain_done = []
    plain_work = 0
    for M, e in zip(Ms, elems):
        r = rp.solve(M, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        plain_done.append(time.perf_counter() - t0)
        plain_work += e * r.iterations
    plain_wall = plain_done[-1]
    achieved = prof["update_bytes"] / (prof["update_ms"] * 1e-3) / 1e9 if prof["update_ms"] > 0 else 0.0
    value = work / wall
    return {
        "workload": "rpca_batch64_uneven", "count": len(Ms), "steps": steps, "warmup": warmup,
        "tol": tol, "maxit": maxit, "elements": int(sum(elems)),
        "iterations_min": int(min(iters)), "iterations_max": int(max(iters)),
        "iterations_mean": float(np.mean(iters)),
        "value": value, "unit": "pixel-frames/s per ALM iter",
        "ms_per_step": wall / steps * 1e3,
        "solves_per_s": len(Ms) * steps / wall,
        # 5 FP32 words per entry and iteration (read X, S, Y; write S, Y) over wall time
        "per_iteration_frac": value * 20.0 / (HBM_PEAK_GBS * 1e9),
        "update_kernels": {"achieved_GBps": achieved, "frac": achieved / HBM_PEAK_GBS,
                           "launches": prof["update_launches"],
                           "measured_on": "one extra step, each launch recording its own HIP "
                                          "start/stop event pair (one stream)"},
        "latency_ms": {"p50": float(np.percentile(walls, 50)) * 1e3,
                       "p99": float(np.percentile(walls, 99)) * 1e3},
        "kernel_timed_step": {"ms": timed_wall * 1e3,
                              **{k: prof[k] for k in ("init_ms", "eig_ms", "update_ms", "finalize_ms")}},
        "plain": {"value": plain_work / plain_wall, "solves_per_s": len(Ms) / plain_wall,
                  "per_iteration_frac": plain_work / plain_wall * 20.0 / (HBM_PEAK_GBS * 1e9),
                  "latency_ms": {"p50": float(np.percentile(plain_done, 50)) * 1e3,
                                 "p99": float(np.percentile(plain_done, 99)) * 1e3}},
    }


def run_batch(args):
    """The 64-window batch as its own bench line."""
    b = batch_measure(args.count, args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": b["value"],
        "unit": "pixel-frames/s per ALM iter",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (64 seeded ultrasound-shaped windows, density 1 bound + 2 free "
                "bubbles per 1300 px^2)",
        "config": {k: b[k] for k in ("workload", "count", "tol", "maxit", "elements",
                                     "iterations_min", "iterations_max", "iterations_mean")},
        "solves_per_s": b["solves_per_s"],
        "latency_ms": b["latency_ms"],
        "roofline": {"bound": "hbm", "achieved": b["update_kernels"]["achieved_GBps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": b["update_kernels"]["frac"],
                     "per_iteration_frac": b["per_iteration_frac"], "traffic": None,
                     "kernel": "update pass, all frame classes (k_wide MFMA tile kernel for the "
                               "classes in tuning.tile_kernel_classes, k_stream register kernel "
                               "for the others)",
                     "launches": b["update_kernels"]["launches"],
                     "measured_on": b["update_kernels"]["measured_on"]},
        "tuning": tuning_summary(),
        "kernel_timed_step": b["kernel_timed_step"],
        "plain": b["plain"],
    }
    print(json.dumps(out), flush=True)


def latency_128x128x20_f64(solves: int = 20) -> dict:
    """The latency workload: one FP64 solve of the seeded 128x128 x 20 window
    (lambda 1/128, tol 1e-7, maxit 500) per call, p50/p99 of the call time."""
    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth import window_128x128x20

    X = window_128x128x20().X()
    m, n = X.shape
    M = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0").t()
    kw = dict(lam=1.0 / 128, tol=1e-7, maxit=500)
    rp.solve(M, **kw)
    torch.cuda.synchronize()
    times, its = [], []
    for _ in range(solves):
        t0 = time.perf_counter()
        r = rp.solve(M, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(r.iterations)
    it = int(np.median(its))
    return {"workload": "rpca_128x128x20_f64_latency", "m": m, "n": n, "dtype": "f64", **kw,
            "solves": solves, "iterations": it, "status": int(r.status),
            "latency_ms": {"p50": float(np.percentile(times, 50)) * 1e3,
                           "p99": float(np.percentile(times, 99)) * 1e3},
            "us_per_iteration": float(np.median(times)) / max(it, 1) * 1e6,
            "value": m * n * it / float(np.median(times)), "unit": "pixel-frames/s per ALM iter"}


def fingerprint(t) -> int:
    """Exact hash of a result's bits (integer sum, independent of order), so a
    served result can be compared with the same window solved alone without
    keeping both in memory."""
    import torch
    flat = t.t().contiguous().view(-1)
    v = flat.view(torch.int32 if flat.dtype == torch.float32 else torch.int64).to(torch.int64)
    w = torch.arange(v.numel(), device=v.device, dtype=torch.int64) % 1000003 + 1
    return int((v * w).sum())


def serve_trace_run(reqs, args, plain: bool, check_every: int, prebuilt=None):
    """Serve `reqs` [(t, side, n, seed)] as they arrive, through the server
    (or, plain=True, one rp.solve per request in arrival order).  Arrived
    requests wait in a client-side FIFO in front of the server's own queue,
    which is kept a few requests deep; latency counts from arrival.  The
    input windows are `prebuilt` (device tensors in arrival order), or are
    built ahead of their arrival, at most 16 windows ahead, so that building
    them does not hold up the server: the host-side draws of a window (up to
    a few tenths of a second of Python for the largest) run in a process
    pool, and a producer thread renders them on a stream of its own.  Returns the completion times, statuses,
    iterations and, for every check_every-th request, a fingerprint of L and
    S."""
    import queue
    import threading

    import torch

    import paper_2506_10257_amd as rp
    from paper_2506_10257_amd.server import Server
    from synth.device import device_window

    dev = torch.device("cuda:0")
    tol, maxit = 1e-6, 1000

    def build(i):
        _, side, n, seed = reqs[i]
        return device_window(side, side, n, seed, dev).view(n, side * side).t()

    halt = threading.Event()
    producer = None
    if prebuilt is not None:
        def take(i, block=True):
            return prebuilt[i]
    else:
        # host-side draws in worker processes (submitted in order, at most 64
        # ahead), device rendering in this thread on a stream of its own
        from concurrent.futures import ProcessPoolExecutor
        from synth.device import render_window, window_geometry

        ready = queue.Queue(maxsize=16)
        side = torch.cuda.Stream(device=dev)
        pool = ProcessPoolExecutor(min(16, len(os.sched_getaffinity(0))))

        def produce():
            try:
                futs = {}
                with torch.cuda.stream(side):
                    for i in range(len(reqs)):
                        for k in range(i, min(i + 64, len(reqs))):
                            if k not in futs:
                                _, sd, nn, seed = reqs[k]
                                futs[k] = pool.submit(window_geometry, sd, sd, nn, seed)
                        _, sd, nn, _ = reqs[i]
                        M = render_window(futs.pop(i).result(), dev).view(nn, sd * sd).t()
                        side.synchronize()
                        while True:
                            if halt.is_set():
                                return
                            try:
                                ready.put((i, M), timeout=0.5)
                                break
                            except queue.Full:
                                pass
            except BaseException as e:  # handed to the consumer, which raises it
                while not halt.is_set():
                    try:
                        ready.put((-1, e), timeout=0.5)
                        break
                    except queue.Full:
                        pass

        producer = threading.Thread(target=produce, name="window-producer", daemon=True)
        producer.start()

        def take(i, block=True):
            """Window i, or None when block is False and it is not built yet."""
            try:
                j, M = ready.get(block=block)
            except queue.Empty:
                return None
            if j < 0:
                raise M
            assert j == i, (j, i)
            return M

    done_at, iters, status, fps = {}, {}, {}, {}

    def record(tag, st, it, L, S, t_done):
        done_at[tag] = t_done
        iters[tag] = it
        status[tag] = st
        if check_every and tag % check_every == 0 and L is not None:
            fps[tag] = (fingerprint(L), fingerprint(S))

    t0 = time.perf_counter()
    note = 10.0
    peak = 0
    try:
        if plain:
            for k, (t, _, _, _) in enumerate(reqs):
                now = time.perf_counter() - t0
                if now >= note:
                    print(f"[serve] plain {now:.0f} s: {k} of {len(reqs)} done", file=sys.stderr, flush=True)
                    note += 10.0
                if now < t:
                    time.sleep(t - now)
                r = rp.solve(take(k), tol=tol, maxit=maxit)
                torch.cuda.synchronize()
                record(k, r.status, r.iterations, r.L, r.S, time.perf_counter() - t0)
                del r
        else:
            srv = Server(rp.RPCA_F32, hbm_budget=int(args.budget_gb * (1 << 30)),
                         max_active=args.max_active, quantum=args.quantum)
            nxt = 0  # next request to hand to the server
            while len(done_at) < len(reqs):
                now = time.perf_counter() - t0
                if now >= note:
                    print(f"[serve] {now:.0f} s: {len(done_at)} of {len(reqs)} done, "
                          f"{nxt} handed over", file=sys.stderr, flush=True)
                    note += 10.0
                left, queued, _, _ = srv.pending()
                while nxt < len(reqs) and reqs[nxt][0] <= now and queued < 8:
                    # with work in the server, a window not built yet waits for the next step
                    M = take(nxt, block=left == 0)
                    if M is None:
                        break
                    srv.submit(M, tag=nxt, tol=tol, maxit=maxit)
                    nxt += 1
                    queued += 1
                    left += 1
                if left == 0:
                    if nxt < len(reqs):
                        time.sleep(max(0.0, reqs[nxt][0] - (time.perf_counter() - t0)))
                    continue
                for c in srv.step():
                    record(c.tag, c.status, c.iterations, c.L, c.S, time.perf_counter() - t0)
                    c.L = c.S = None
            peak = srv.peak_bytes()
            srv.close()
    finally:
        halt.set()
        if producer is not None:
            producer.join()
            pool.shutdown(cancel_futures=True)
    wall = time.perf_counter() - t0
    return done_at, iters, status, fps, wall, peak


def serve_summary(reqs, done_at, iters, status, wall):
    import numpy as np
    lat = np.array([done_at[k] - reqs[k][0] for k in range(len(reqs))])
    elems = [side * side * n for (_, side, n, _) in reqs]
    work = sum(elems[k] * iters[k] for k in range(len(reqs)))
    st = list(status.values())
    return {"requests": len(reqs), "wall_s": wall, "solves_per_s": len(reqs) / wall,
            "value": work / wall, "per_iteration_frac": work / wall * 20.0 / (HBM_PEAK_GBS * 1e9),
            "latency_ms": {"p50": float(np.percentile(lat, 50)) * 1e3,
                           "p99": float(np.percentile(lat, 99)) * 1e3},
            "statuses": {str(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
            "iterations_mean": float(np.mean(list(iters.values())))}


def run_serve(args):
    """Poisson arrivals of square windows (256-1024 px sides, 10/20/40/100
    frames, FP32, tol 1e-6, maxit 1000) served by the continuous-batching
    server.  Two parts:
      * the full trace at args.rate for args.duration s through the server
        (its windows built ahead of arrival by a producer thread, so the
        client's input generation does not hold the server up); every
        args.check_every-th served result is compared bit for bit with the
        same window solved alone (plain path);
      * a sustainable arrival rate (args.sustain_rate, 3 req/s by default,
        about 60% of what the server completes on this mix), where the
        server's latency measures service rather than queueing, through the
        server and through the plain path (one solve per call, first come
        first served) on the same trace, with every window built before the
        clock starts; --sustain-only runs this part alone.
    The plain path is not run on the full trace: at its capacity (about a
    third of the server's) the 60 s trace would take the better part of an
    hour."""
    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth import serve_trace

    frames = tuple(int(f) for f in args.serve_frames.split(","))

    def trace_of(rate, duration, seed):
        rng = np.random.default_rng(55)
        out = []
        for (t, side, n, sd) in serve_trace(rate_hz=rate, duration_s=duration, seed=seed):
            if n not in frames:
                n = int(frames[rng.integers(len(frames))])
            out.append((t, side, n, sd))
        return out

    reqs = trace_of(args.rate, args.duration, 5)
    elems = sum(side * side * n for (_, side, n, _) in reqs)
    print(f"[serve] {len(reqs)} requests over {args.duration:.1f} s, {elems / 1e9:.2f} G elements",
          file=sys.stderr, flush=True)
    from synth.device import device_window
    w0 = device_window(64, 64, 10, 1, torch.device("cuda:0")).view(10, 4096).t()
    rp.solve(w0, tol=1e-6, maxit=5)
    torch.cuda.synchronize()

    full, checked, equal = None, 0, 0
    if not args.sustain_only:
        done_at, iters, status, fps, wall, peak = serve_trace_run(reqs, args, False, args.check_every)
        full = serve_summary(reqs, done_at, iters, status, wall)
        full["peak_admitted_gb"] = peak / 2 ** 30
        print(f"[serve] full trace: {full['solves_per_s']:.2f} solves/s, p99 {full['latency_ms']['p99']:.0f} ms",
              file=sys.stderr, flush=True)

        # bitwise check of the sampled served results against the same windows alone
        from synth.device import device_window as dw
        checked = equal = 0
        for tag, (fL, fS) in sorted(fps.items()):
            _, side, n, seed = reqs[tag]
            M = dw(side, side, n, seed, torch.device("cuda:0")).view(n, side * side).t()
            r = rp.solve(M, tol=1e-6, maxit=1000)
            checked += 1
            equal += int(fingerprint(r.L) == fL and fingerprint(r.S) == fS and
                         r.iterations == iters[tag] and r.status == status[tag])
            del r, M
            if checked % 50 == 0:
                print(f"[serve] bitwise check: {equal} of {checked} equal so far", file=sys.stderr, flush=True)
        print(f"[serve] bitwise check: {equal} of {checked} equal", file=sys.stderr, flush=True)

    # a sustainable arrival rate: server and plain path on the same trace
    # (its windows are built before the clock starts, so the latencies are
    # those of the server and of the plain path alone)
    sreqs = trace_of(args.sustain_rate, args.sustain_duration, 6)
    dev = torch.device("cuda:0")
    swin = [device_window(side, side, n, seed, dev).view(n, side * side).t()
            for (_, side, n, seed) in sreqs]
    torch.cuda.synchronize()
    d2, i2, s2, _, w2, p2 = serve_trace_run(sreqs, args, False, 0, prebuilt=swin)
    sus = serve_summary(sreqs, d2, i2, s2, w2)
    d3, i3, s3, _, w3, _ = serve_trace_run(sreqs, args, True, 0, prebuilt=swin)
    del swin
    sus_plain = serve_summary(sreqs, d3, i3, s3, w3)
    out = {
        "metric": METRIC,
        "value": full["value"] if full else sus["value"],
        "unit": "pixel-frames/s per ALM iter",
        "n_gpus": 1, "steps": len(reqs if full else sreqs), "warmup": 1,
        "ms_per_step": (full or sus)["wall_s"] / len(reqs if full else sreqs) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Poisson arrivals; square windows 256..1024 px, device-built "
                "ultrasound-shaped frames)",
        "config": {"workload": "rpca_serve_poisson", "rate_hz": args.rate,
                   "duration_s": args.duration, "requests": len(reqs), "frames": list(frames),
                   "tol": 1e-6, "maxit": 1000, "max_active": args.max_active,
                   "quantum": args.quantum, "hbm_budget_gb": args.budget_gb},
        "served": full,
        "bitwise_vs_alone": {"sample": f"every {args.check_every}th request", "checked": checked,
                             "equal": equal},
        "sustainable": {"rate_hz": args.sustain_rate, "duration_s": args.sustain_duration,
                        "served": sus, "plain": sus_plain},
        "tuning": tuning_summary(),
    }
    print(json.dumps(out), flush=True)


def run_precision(args):
    """1024x1024x40 window (15 dB): the FP32 path against the split-BF16
    contraction modes (two- and three-way splits).  Throughput of full solves (tol 1e-6, maxit 1000) for
    both, and the error of each against the FP64 oracle at a fixed iteration
    count (the oracle's full solve of this window takes hours on a host)."""
    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth import window_1024x1024x40
    from oracle import rpca, rel_fro, dice, bound_threshold

    dev = torch.device("cuda:0")
    w = window_1024x1024x40()
    X = w.X()
    m, n = X.shape
    M = torch.from_numpy(np.ascontiguousarray(X.T.astype(np.float32))).to(dev).t()
    tol, maxit = 1e-6, 1000
    modes = {"f32": rp.RPCA_GRAM_DEFAULT, "bf16x3": rp.RPCA_GRAM_BF16X3,
             "bf16x6": rp.RPCA_GRAM_BF16X6}
    out_modes = {}
    for name, gm in modes.items():
        for _ in range(args.warmup):
            rp.solve(M, tol=tol, maxit=maxit, gram_mode=gm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for _ in range(args.steps):
            r = rp.solve(M, tol=tol, maxit=maxit, gram_mode=gm)
            torch.cuda.synchronize()
            iters += r.iterations
        wall = time.perf_counter() - t0
        out_modes[name] = {"value": m * n * iters / wall, "ms_per_solve": wall / args.steps * 1e3,
                           "iterations": r.iterations, "status": r.status}
        print(f"[precision] {name}: {out_modes[name]}", file=sys.stderr, flush=True)
    # error against the oracle at a fixed iteration count
    K = args.parity_iters
    ref = rpca(X, tol=0.0, maxit=K)
    theta = bound_threshold(w.L_gt, w.bound_mask)
    for name, gm in modes.items():
        r = rp.solve(M, tol=0.0, maxit=K, gram_mode=gm)
        Lh = r.L.t().contiguous().cpu().numpy().T.astype(np.float64)
        Sh = r.S.t().contiguous().cpu().numpy().T.astype(np.float64)
        out_modes[name]["error_vs_oracle_at_k"] = {
            "k": K, "relL": rel_fro(Lh, ref.L), "relS": rel_fro(Sh, ref.S),
            "dice": dice(Lh >= theta, ref.L >= theta)}
    f32 = out_modes["f32"]
    out = {
        "metric": METRIC,
        "value": f32["value"],
        "unit": "pixel-frames/s per ALM iter",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f32["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ultrasound-shaped window: rank-2 drifting speckle, 800 bound + "
                "1600 free bubbles on 24 vessels, 15 dB SNR)",
        "config": {"workload": "rpca_1024x1024x40_precision", "m": m, "n": n, "tol": tol,
                   "maxit": maxit},
        "modes": out_modes,
        "tuning": tuning_summary(),
    }
    print(json.dumps(out), flush=True)


def run_sliding(args):
    """Sliding 20-frame windows (step 5) over a sequence of square frames: every window
    solved from zero against every window started from the previous window's
    S and Y shifted by the step (the real-time use of the method)."""
    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth import make_window, density_counts

    dev = torch.device("cuda:0")
    n, step, K = 20, 5, args.windows
    side = args.sliding_side
    nb_, nf_, nv_ = density_counts(side, side)
    w = make_window(side, side, n + step * (K - 1), nb_, nf_, nv_, 20.0, 21)
    seq = torch.from_numpy(np.ascontiguousarray(w.X().T.astype(np.float32))).to(dev).t()
    m = seq.shape[0]
    tol, maxit = 1e-6, 1000
    wins = [seq[:, j * step: j * step + n] for j in range(K)]
    rp.solve(wins[0], tol=tol, maxit=5)
    torch.cuda.synchronize()

    def run(warm):
        times, iters, outs = [], [], []
        prev = None
        for M in wins:
            S0 = Y0 = None
            if warm and prev is not None:
                S0 = torch.zeros_like(M)
                Y0 = torch.zeros_like(M)
                S0[:, : n - step].copy_(prev.S[:, step:])
                Y0[:, : n - step].copy_(prev.Y[:, step:])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = rp.solve(M, tol=tol, maxit=maxit, S0=S0, Y0=Y0, return_Y=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters.append(r.iterations)
            outs.append(r.L)
            prev = r
        return times, iters, outs

    ct, ci, cl = run(False)
    wt, wi, wl = run(True)
    rel = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(wl, cl))
    work = sum(m * n * k for k in wi)
    out = {
        "metric": METRIC,
        "value": work / sum(wt),
        "unit": "pixel-frames/s per ALM iter",
        "n_gpus": 1, "steps": K, "warmup": 1,
        "ms_per_step": sum(wt) / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ultrasound-shaped sequence, 1 bound + 2 free bubbles per "
                "1300 px^2, 20 dB)",
        "config": {"workload": f"rpca_sliding_{side}x{side}_w20_s5", "windows": K, "frames": n,
                   "step": step, "tol": tol, "maxit": maxit},
        "warm": {"windows_per_s": K / sum(wt), "iterations_mean": float(np.mean(wi)),
                 "latency_ms": {"p50": float(np.percentile(wt, 50)) * 1e3,
                                "p99": float(np.percentile(wt, 99)) * 1e3}},
        "cold": {"windows_per_s": K / sum(ct), "iterations_mean": float(np.mean(ci)),
                 "latency_ms": {"p50": float(np.percentile(ct, 50)) * 1e3,
                                "p99": float(np.percentile(ct, 99)) * 1e3}},
        "max_rel_L_warm_vs_cold": rel,
        "tuning": tuning_summary(),
    }
    print(json.dumps(out), flush=True)


def run_postproc(args):
    """The steps around the solve on a 1024x1024 x 132-frame FP32 sequence
    (the paper's reference window length): frame correlation, frame
    selection, 20-frame moving average, Dice and RMSE.  Each is one HBM
    pass; reported as algorithmic bytes / wall time against the HBM peak."""
    import numpy as np
    import torch

    import paper_2506_10257_amd.postproc as pp
    from synth.device import device_window

    dev = torch.device("cuda:0")
    side, n, W = 1024, 132, 20
    x = device_window(side, side, n, 31, dev)
    M = x.view(n, side * side).t()
    m = M.shape[0]
    B = M.clone()
    torch.cuda.synchronize()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    keep = pp.frame_keep(pp.frame_correlation(M), 0.8)
    steps = {
        "frame_correlation": (lambda: pp.frame_correlation(M), 4.0 * m * n),
        "frame_select": (lambda: pp.frame_select(M, keep), 8.0 * m * int(keep.sum())),
        "moving_average_w20": (lambda: pp.moving_average(M, W), 4.0 * m * n + 4.0 * m * (n - W + 1)),
        "dice": (lambda: pp.dice(M, 1.0, B, 1.0), 8.0 * m * n),
        "rmse": (lambda: pp.rmse(M, B), 8.0 * m * n),
    }
    res = {}
    for name, (fn, nbytes) in steps.items():
        t = timed(fn, args.steps)
        res[name] = {"ms": t * 1e3, "GB/s": nbytes / t / 1e9, "frac_of_hbm_peak": nbytes / t / 1e9 / HBM_PEAK_GBS}
        print(f"[postproc] {name}: {res[name]}", file=sys.stderr, flush=True)
    total = sum(v["ms"] for v in res.values())
    out = {
        "metric": "pixel-frames/s through correlation, selection, moving average, Dice and RMSE",
        "value": m * n / (total * 1e-3), "unit": "pixel-frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": total,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (device-built ultrasound-shaped 1024x1024 x 132-frame sequence)",
        "config": {"workload": "postproc_1024x1024x132", "W": W, "kept": int(keep.sum())},
        "kernels": res,
    }
    print(json.dumps(out), flush=True)


def run_frames132(args):
    """One FP32 solve of a 512x512 x 132-frame window (the paper's reference
    window length): 144-frame tile kernel and the eigensolver with V in
    device memory.  Throughput of the graph path, then a kernel-timed repeat
    for the eigensolve / update split and the update kernel's roofline."""
    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth.device import device_window

    dev = torch.device("cuda:0")
    side, n = 512, 132
    M = device_window(side, side, n, 132, dev).view(n, side * side).t()
    m = M.shape[0]
    tol, maxit = 1e-6, args.maxit132
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        rp.solve(M, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(args.steps):
        r = rp.solve(M, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        iters.append(r.iterations)
        print(f"[frames132] solve: {r.iterations} iterations, status {r.status}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    rp.rpca_profile_read(reset=True)
    rp.rpca_profile_enable(True)
    rp.solve(M, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    rp.rpca_profile_enable(False)
    prof = rp.rpca_profile_read(reset=True)
    upd_ms = prof["update_ms"] / max(prof["update_launches"], 1)
    eig_ms = prof["eig_ms"] / max(prof["eig_launches"], 1)
    bytes_per_launch = prof["update_bytes"] / max(prof["update_launches"], 1)
    achieved = bytes_per_launch / (upd_ms * 1e-3) / 1e9 if upd_ms > 0 else 0.0
    out = {
        "metric": METRIC, "value": m * n * sum(iters) / wall, "unit": "pixel-frames/s per ALM iter",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (device-built ultrasound-shaped 512x512 x 132-frame window, batch density)",
        "config": {"workload": "rpca_512x512x132_single_solve", "m": m, "n": n, "tol": tol,
                   "maxit": maxit, "iterations": iters},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "per_iteration_achieved": m * n * sum(iters) / wall * 20.0 / 1e9,
                     "per_iteration_frac": m * n * sum(iters) / wall * 20.0 / (HBM_PEAK_GBS * 1e9),
                     "kernel": "k_wide<float, 144, 1, 0>",
                     "bytes_per_launch": bytes_per_launch, "mean_launch_us": upd_ms * 1e3,
                     "launches": prof["update_launches"],
                     "measured_on": "one repeated solve, each launch recording its own HIP "
                                    "start/stop event pair"},
        "eig_us_per_iter": eig_ms * 1e3,
        "tuning": tuning_summary(),
    }
    print(json.dumps(out), flush=True)


def run_copycal(args):
    """A plain device copy of a known size (256 MiB), repeated: the reference
    that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy_256MiB", "bytes_read": nbytes, "bytes_written": nbytes,
                      "copies": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--workload", choices=["single", "batch", "serve", "precision", "sliding",
                                           "postproc", "frames132", "copycal"], default="single")
    ap.add_argument("--windows", type=int, default=9, help="sliding: windows in the sequence")
    ap.add_argument("--sliding-side", type=int, default=256, help="sliding: frame side (px)")
    ap.add_argument("--parity-iters", type=int, default=5,
                    help="precision: iterations compared with the oracle")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in tuning choices instead of measuring them first")
    ap.add_argument("--count", type=int, default=64, help="windows in the batch workload")
    ap.add_argument("--rate", type=float, default=50.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: trace length (s)")
    ap.add_argument("--check-every", type=int, default=10,
                    help="serve: every k-th served result is compared bit for bit with the window solved alone")
    ap.add_argument("--sustain-rate", type=float, default=3.0,
                    help="serve: arrival rate of the second, sustainable-rate trace")
    ap.add_argument("--sustain-duration", type=float, default=40.0,
                    help="serve: length of the sustainable-rate trace (s)")
    ap.add_argument("--sustain-only", action="store_true",
                    help="serve: run only the sustainable-rate trace (server and plain path)")
    ap.add_argument("--serve-frames", default="10,20,40,100", help="serve: allowed frame counts")
    ap.add_argument("--max-active", type=int, default=48, help="serve: active solves at most")
    ap.add_argument("--quantum", type=int, default=16, help="serve: iterations per step")
    ap.add_argument("--budget-gb", type=float, default=160.0, help="serve: admission budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="single: skip the 128x128x20 FP64 latency and the 64-window batch records")
    ap.add_argument("--maxit132", type=int, default=300, help="frames132: iteration cap")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the RPCA path runs on a single MI355X "
              "(solves would shard across GPUs as whole requests; only the one-GPU path exists)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "copycal":
        run_copycal(args)
        return
    if not args.no_autotune:
        # every workload runs on tuned launch choices (eigensolver workgroup
        # sizes, kernel per frame class, tile rows), chosen on a 262144-row
        # (512 x 512) window before anything is timed
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        import paper_2506_10257_amd as rp
        dt = rp.RPCA_F64 if args.dtype == "f64" and args.workload == "single" else rp.RPCA_F32
        t0 = time.perf_counter()
        rc = rp.rpca_autotune(dt, 262144)
        if rc != rp.RPCA_OK:
            print(f"autotune failed ({rc}): {rp.rpca_last_error()}", file=sys.stderr)
            sys.exit(1)
        print(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return
    if args.workload == "sliding":
        run_sliding(args)
        return
    if args.workload == "postproc":
        run_postproc(args)
        return
    if args.workload == "frames132":
        run_frames132(args)
        return

    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth import window_512x512x20

    dev = torch.device("cuda:0")
    w = window_512x512x20()
    X = w.X()
    m, n = X.shape
    lam, tol, maxit = 1.0 / 512.0, 1e-6, 1000
    npdt = np.float32 if args.dtype == "f32" else np.float64
    M = torch.from_numpy(np.ascontiguousarray(X.T.astype(npdt))).to(dev).t()
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        rp.solve(M, lam=lam, tol=tol, maxit=maxit)
    torch.cuda.synchronize()

    # Timed region: the production path (graph-captured iteration chunks).
    times, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        r = rp.solve(M, lam=lam, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters.append(r.iterations)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    # Kernel timing: the same steps again, every launch recording a HIP
    # start/stop event pair of its own on the launching stream (direct
    # launches, since per-launch events cannot be read back from a replayed
    # graph chunk).
    rp.rpca_profile_read(reset=True)
    rp.rpca_profile_enable(True)
    ktimes = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        rp.solve(M, lam=lam, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        ktimes.append(time.perf_counter() - t0)
    rp.rpca_profile_enable(False)
    prof = rp.rpca_profile_read(reset=True)

    value = sum(m * n * k for k in iters) / wall
    upd_ms = prof["update_ms"] / max(prof["update_launches"], 1)
    bytes_per_launch = prof["update_bytes"] / max(prof["update_launches"], 1)
    achieved = bytes_per_launch / (upd_ms * 1e-3) / 1e9 if upd_ms > 0 else 0.0
    # Which update kernel ran: the register kernel of the 20-frame class, or
    # the MFMA tile kernel (32-frame tile) when the tuner chose it for that
    # class.  The committed counter summary covers the register kernel only.
    # Names as rocprofv3 prints them: k_stream<T, NB, MODE, MT> (MODE 1 =
    # update, MT = several tiles per workgroup), k_wide<T, NB, MODE, PREC>.
    ts = tuning_summary()
    tiled = args.dtype == "f32" and 20 in ts["tile_kernel_classes"]
    if tiled:
        kname, traffic = "k_wide<float, 32, 1, 0>", None
    else:
        mt = ts[f"reg_tiles_{args.dtype}"].get("20", 1) > 1
        kname = f"k_stream<{'float' if args.dtype == 'f32' else 'double'}, 20, 1, {'true' if mt else 'false'}>"
        traffic = measured_traffic() if args.dtype == "f32" and not mt else None
    lat = np.array(times) * 1e3
    wbytes = 4 if args.dtype == "f32" else 8
    per_iter_gbs = value * 5 * wbytes / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pixel-frames/s per ALM iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded ultrasound-shaped window: rank-2 drifting speckle, "
                "200 bound + 400 free bubbles on 6 vessels, 20 dB SNR)",
        "config": {"workload": "rpca_512x512x20_single_solve", "m": m, "n": n,
                   "lambda": lam, "tol": tol, "maxit": maxit,
                   "iterations": int(np.median(iters))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     # the whole iteration (eigensolve, update and reduction in
                     # series): 5 words per entry and iteration over solve wall time
                     "per_iteration_achieved": per_iter_gbs,
                     "per_iteration_frac": per_iter_gbs / HBM_PEAK_GBS,
                     "kernel": kname,
                     "bytes_per_launch": bytes_per_launch, "mean_launch_us": upd_ms * 1e3,
                     "launches": prof["update_launches"],
                     "measured_on": "the same steps repeated, each launch recording its own HIP "
                                    "start/stop event pair"},
        "phase_ms_per_solve": {k: prof[k] / max(prof["solves"], 1)
                               for k in ("init_ms", "eig_ms", "update_ms", "finalize_ms")},
        "tuning": tuning_summary(),
        "kernel_timed_steps": {"ms_per_step": float(np.mean(ktimes)) * 1e3},
        "paper_context": paper_context(args.dtype),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, lam)
    if not args.no_extra:
        out["latency_128x128x20_f64"] = latency_128x128x20_f64()
        print(f"[bench] latency workload: {out['latency_128x128x20_f64']['latency_ms']}",
              file=sys.stderr, flush=True)
        out["batch"] = batch_measure(64, 3, 1)
    print(json.dumps(out), flush=True)


def paper_context(dtype: str) -> dict:
    """The paper reports whole-decomposition times only: 0.2 s on average for
    its 338 x 260-pixel x 20-frame in vivo windows on one RTX 3090 (PyTorch
    with CUDA, precision, iteration count and lambda not stated; stopping at
    1e-9).  Context, not a target: this library's solve time for a synthetic
    window of that size at the workloads' tol (1e-6, maxit 1000)."""
    import numpy as np
    import torch

    import paper_2506_10257_amd as rp
    from synth.device import device_window

    H, W, n = 260, 338, 20
    tdt = torch.float32 if dtype == "f32" else torch.float64
    M = device_window(H, W, n, 338, torch.device("cuda:0"), dtype=tdt).view(n, H * W).t()
    rp.solve(M, tol=1e-6, maxit=1000)
    torch.cuda.synchronize()
    times, its = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        r = rp.solve(M, tol=1e-6, maxit=1000)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(r.iterations)
    return {"paper_solve_s": 0.2, "paper_hardware": "1x NVIDIA RTX 3090, PyTorch with CUDA",
            "paper_window": "338x260 px x 20 frames (87880 x 20), in vivo",
            "this_solve_s": float(np.median(times)), "this_iterations": int(np.median(its)),
            "this_window": "synthetic 338x260 px x 20 frames, tol 1e-6, maxit 1000",
            "dtype": dtype}


if __name__ == "__main__":
    main()
