"""Serving front end: replays a request stream (arrival times, microstructure,
phase parameters, load steps) against the library's continuous-batching
server and reports throughput and latency.

Microstructures are generated on the host before the replay (in worker
processes: the 1000-request stream holds ~2.7e9 voxels); the replay then
submits each request at its arrival time and polls results as they finish.
Latency is measured on the server's clock from the scheduled arrival to the
moment the request's last load step is done and its result is available.
"""
from __future__ import annotations

import multiprocessing
import time

import numpy as np

from . import inputs


def prepare_fields(reqs, workers: int = 8):
    """Phase fields of all requests (uint8 arrays), generated in a pool of
    spawned worker processes (call before the GPU is initialised)."""
    if workers <= 1:
        return [inputs.request_phase_field(q) for q in reqs]
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(workers) as pool:
        return pool.map(inputs.request_phase_field, reqs, chunksize=2)


def _drain(srv, want, timeout):
    got = {}
    t0 = time.perf_counter()
    while len(got) < want:
        for r in srv.poll():
            got[r["id"]] = r
        if time.perf_counter() - t0 > timeout:
            raise TimeoutError(f"{want - len(got)} requests unfinished after {timeout} s")
        time.sleep(0.0005)
    return got


def replay(reqs, fields, sequential=False, saturate=False, budget_bytes=200e9,
           max_batch_points=0, timeout=600.0):
    """Run the stream through a fresh server. saturate=True submits every
    request at time zero (throughput at full load); otherwise each request is
    submitted at its arrival time. Returns a dict of statistics."""
    from . import api
    srv = api.Server(int(budget_bytes), max_batch_points=max_batch_points, sequential=sequential)
    try:
        # warm-up: module load and first launch outside the measurement
        w = reqs[0]
        srv.submit(fields[0][:4096], w.phases, 1, w.E_final, w.noise_std, 1, h=w.h)
        _drain(srv, 1, timeout)
        st0 = srv.stats()
        base = srv.clock()
        t_start = time.perf_counter()
        ids = []
        got = {}
        for q, ph in zip(reqs, fields):
            if not saturate:
                while True:
                    delay = q.arrival - (time.perf_counter() - t_start)
                    if delay <= 0:
                        break
                    for r in srv.poll():
                        got[r["id"]] = r
                    time.sleep(min(delay, 0.0005))
            arrival = base + (0.0 if saturate else q.arrival)
            ids.append(srv.submit(ph, q.phases, q.steps, q.E_final, q.noise_std, q.seed, h=q.h,
                                  arrival=arrival))
        rest = _drain(srv, len(ids) - len(got), timeout)
        got.update(rest)
        st1 = srv.stats()
    finally:
        srv.close()
    res = [got[i] for i in ids]
    failed = sum(r["status"] != 0 for r in res)
    lat = np.array([r["t_done"] - r["t_arrival"] for r in res])
    end = max(r["t_done"] for r in res)
    updates = sum(q.n * q.steps for q in reqs)
    makespan = end - base
    return {
        "mode": "sequential" if sequential else "batched",
        "arrivals": "all at t=0" if saturate else "scheduled",
        "requests": len(reqs),
        "updates": int(updates),
        "makespan_s": makespan,
        "throughput": updates / makespan,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "launches": int(st1["launches"] - st0["launches"]),
        "gpu_busy_s": float(st1["busy_s"] - st0["busy_s"]),
        "nonconverged_points": int(sum(r["nonconverged"] for r in res)),
        "failed_requests": int(failed),
    }
