"""Benchmark: FP64 material-point updates/s of one implicit-Euler GSM
evaluation batch on the 256^3 fibre microstructure (one MI355X).

A step is one call of the whole per-point path (load eps, a_n, phase; AD
residual; Newton with AD Hessian and Cholesky; stress and a_{n+1} stores)
over all 256^3 points, inputs resident in HBM. Timed with events on the
stream the kernels run on. Prints one JSON line.

Roofline: the path streams 193 B per point (reads eps, a_n: 96 B, phase:
1 B; writes sigma, a_{n+1}: 96 B) against 8 TB/s HBM; the dominant kernel's
achieved algorithmic bandwidth is reported as the roofline fraction.
The CPU baseline is the oracle (plain C, OpenMP) timed on a bounded prefix
of the same batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 material-point updates/s at 256^3 (% roofline); served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BYTES_PER_POINT = 6 * 8 + 6 * 8 + 1 + 6 * 8 + 6 * 8          # 193
BYTES_PER_POINT_TANGENT = BYTES_PER_POINT + 36 * 8            # 481
# the conventional entry point also writes its per-point iteration count
BYTES_PER_POINT_CONVENTIONAL = BYTES_PER_POINT + 4             # 197
# FP32: float fields, 36 float tangent components
BYTES_PER_POINT_F32 = 4 * 24 + 1                               # 97
BYTES_PER_POINT_F32_TANGENT = BYTES_PER_POINT_F32 + 36 * 4     # 241
# adaptive schemes: eps_n, eps_{n+1}, a_n and the phase in; sigma, a_{n+1}
# and the accepted step count out
BYTES_PER_POINT_RK = 3 * 6 * 8 + 1 + 2 * 6 * 8 + 4             # 245
BYTES_PER_POINT_RK_TANGENT = BYTES_PER_POINT_RK + 36 * 8       # 533


# HBM bytes per launch of the forward kernel measured with rocprofv3
# FETCH_SIZE / WRITE_SIZE (scaled by a 1 GiB copy calibration), keyed by the
# hash of the kernel sources they were taken on; a changed kernel reports
# traffic null until it is measured again.
# Algorithmic HBM bytes per voxel and iteration of the basic scheme on grids
# with 128 x 128 planes and cold Newton starts: the half spectrum of six
# components is 6 x 65 x 16 B per 128 voxels (48.75 B); sweep 145 (reads eps,
# a_n and the phase, writes tau), forward plane transforms 96.75 (tau in, half
# spectrum out), z transforms with the Green operator 97.5, inverse plane
# transforms with the strain update 144.75 (half spectrum and eps in, eps out).
MS_HALF_SPECTRUM_BYTES = 6 * 65 * 16 / 128
MS_BYTES_PER_VOXEL = ((48 + 48 + 1 + 48) + (48 + MS_HALF_SPECTRUM_BYTES)
                      + 2 * MS_HALF_SPECTRUM_BYTES + (MS_HALF_SPECTRUM_BYTES + 48 + 48))   # 484
MEASURED_TRAFFIC = {"f48d9ced49bd27d1": 3.351e9}
# Executed FP64 FLOP per point of the forward kernel on the 256^3 batch
# (rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes / points), same keying.
MEASURED_FP64_FLOP_PER_POINT = {"f48d9ced49bd27d1": 1119.0}
KERNEL_SOURCES = ["automat.hip", "ad.hpp", "fastmath.hpp", "linalg6.hpp", "msgsm.hpp",
                  "gsm_point.hpp", "gsm_kernel.hpp"]


def kernel_source_hash():
    """Hash of the forward kernel's sources and of the compiler command line
    they are built with (the flags change the code too)."""
    import hashlib
    from paper_2006_04391_amd import build
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2006_04391_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    flags = build._flags()
    # include paths differ from one checkout to another; the rest is the code
    kept = [f for k, f in enumerate(flags) if f != "-I" and (k == 0 or flags[k - 1] != "-I")]
    h.update(" ".join(kept).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hbm_roofline(bytes_per_point, n, ms):
    """HBM roofline of a leg: its algorithmic bytes per point times the
    points of one launch over the measured time per launch."""
    gbs = bytes_per_point * n / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "bytes_per_point": bytes_per_point, "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def time_calls(fn, steps, warmup, stream):
    """Time `steps` calls back to back (events on the launch stream around the
    whole loop: total_ms; host clock: wall), then the same number of calls
    with events around each (each, per-launch durations)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    per = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        per.append((e0, e1))
    torch.cuda.synchronize()
    each = [a.elapsed_time(b) for a, b in per]
    return total_ms, each, wall


def latency_c0(dev, calls=200):
    """The 4096-point parity set (70 % viscoplastic matrix, 30 % elastic
    inclusion, h = 0.1 s): latency of one evaluation call, inputs resident
    on the device. end_to_end: the Python call through the binding plus a
    stream synchronization, host clock; kernel: events around the launch."""
    import torch
    from paper_2006_04391_amd import api, inputs
    ps = inputs.points_c0()
    eps = torch.from_numpy(ps.eps).to(dev)
    a_old = torch.from_numpy(ps.a_old).to(dev)
    phase = torch.from_numpy(ps.phase).to(dev)
    sigma = torch.empty_like(eps)
    a_new = torch.empty_like(a_old)
    tan = torch.empty((36, ps.n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {"workload": "4096 points (2867 viscoplastic matrix, 1229 elastic inclusion), "
                       "h = 0.1 s, tol 1e-12, inputs resident on the device"}
    for key, tangent in (("no_tangent", False), ("tangent", True)):
        def call():
            api.evaluate(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                         sigma_out=sigma, a_out=a_new, tangent=tangent,
                         tangent_out=tan if tangent else None)
        for _ in range(20):
            call()
        torch.cuda.synchronize()
        host = []
        for _ in range(calls):
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            host.append(time.perf_counter() - t0)
        _, each, _ = time_calls(call, calls, 5, stream)
        out[key] = {"end_to_end_us_median": float(np.median(host)) * 1e6,
                    "end_to_end_us_p99": float(np.percentile(host, 99)) * 1e6,
                    "kernel_us_median": float(np.median(each)) * 1e3}
        log(f"[bench] 4096 points ({key}): end-to-end {np.median(host) * 1e6:.1f} us, "
            f"kernel {np.median(each) * 1e3:.1f} us")
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ps, target_s=3.0):
    """The oracle (plain C, gcc -O3, no fast-math, OpenMP static schedule, one
    point per iteration) on a prefix of the 256^3 batch: the compute call
    alone, median of three runs, on all host threads and on one. The prefix
    grows until one all-thread run takes about target_s; the one-thread
    sample is that prefix divided by the thread count."""
    import oracle
    threads = oracle.num_threads()

    def sample(m):
        return (np.ascontiguousarray(ps.eps[:, :m]), np.ascontiguousarray(ps.a_old[:, :m]),
                np.ascontiguousarray(ps.phase[:m]))

    def run(eps, a_old, phase):
        t0 = time.perf_counter()
        oracle.evaluate(eps, a_old, phase, ps.phases, h=ps.h, tol=ps.tol, max_iter=ps.max_iter)
        return time.perf_counter() - t0

    def median3(m):
        """Median of three runs, each of as many passes over the sample as
        make up about target_s; returns (seconds per pass, run times, passes)."""
        eps, a_old, phase = sample(m)
        t1 = run(eps, a_old, phase)
        reps = max(1, int(round(target_s / max(t1, 1e-3))))
        ts = []
        for _ in range(3):
            ts.append(sum(run(eps, a_old, phase) for _ in range(reps)))
        return float(np.median(ts)) / reps, ts, reps

    m = 1 << 18
    while True:
        m = min(m, ps.n)
        t, ts, reps = median3(m)
        if t >= target_s or m == ps.n:
            break
        m = min(ps.n, int(m * max(2.0, 1.2 * target_s / max(t, 1e-3))))
    m1 = max(1 << 14, m // threads)
    oracle.set_num_threads(1)
    try:
        t1, ts1, reps1 = median3(m1)
    finally:
        oracle.set_num_threads(threads)
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return dict(value=m / t, unit="updates/s", cores=threads, kind="oracle",
                cpu_model=cpu_model(), nproc=nproc, one_core_value=m1 / t1,
                sample=f"first {m} of {ps.n} points of the 256^3 fibre batch (one core: first "
                       f"{m1}), no tangent, compute call only, median of 3 runs of {reps} "
                       f"(one core: {reps1}) passes ({', '.join(f'{x:.2f}' for x in ts)} s on "
                       f"{threads} threads; {', '.join(f'{x:.2f}' for x in ts1)} s on 1 thread)")


def ms_bench(steps, N=128, h=0.1, tol=1e-6):
    """The basic scheme on the 128^3 sphere microstructure (20 %, r = 6):
    uniaxial strain path E(t) = 1e-3 t e11, `steps` steps of h, fixed-point
    tolerance 1e-6; wall time of all steps with the fields resident."""
    import torch
    from paper_2006_04391_amd import api, inputs
    phase = torch.from_numpy(inputs.sphere_phase(N, seed=2)).cuda()
    n = N ** 3
    # cold Newton starts: with these mildly nonlinear parameters a warm start
    # saves fewer updates than its extra traffic costs
    ms = api.MS((N, N, N), inputs.config_phases(), tol=tol, max_iter=5000, warm_start=False)
    eps = torch.zeros((6, n), dtype=torch.float64, device="cuda")
    a = torch.zeros_like(eps)
    ms.step(phase, [0.0] * 6, h, eps, a)       # warm-up (plans, modules)
    eps.zero_()
    a.zero_()
    ms.set_macro([0.0] * 6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    mean = None
    for k in range(1, steps + 1):
        mean, it, _ = ms.step(phase, [1e-3 * h * k, 0, 0, 0, 0, 0], h, eps, a)
        iters.append(it)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms.close()
    total = sum(iters)
    log(f"[bench] MS {N}^3: {steps} steps, {total} iterations, {wall:.2f} s, "
        f"{wall / total * 1e3:.3f} ms/iteration")
    return {"workload": f"Moulinec-Suquet basic scheme, {N}^3 periodic spheres (20 %, r=6), "
                        f"uniaxial strain rate 1e-3/s, {steps} steps of h={h} s, tol {tol}, "
                        f"cold Newton starts",
            "wall_s": wall, "iterations": iters, "ms_per_iteration": wall / total * 1e3,
            "sweep_updates_per_s": total * n / wall, "sigma_mean_last": mean,
            "roofline": {"bound": "hbm", "bytes_per_voxel_iteration": MS_BYTES_PER_VOXEL,
                         "achieved": MS_BYTES_PER_VOXEL * n * total / wall / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": MS_BYTES_PER_VOXEL * n * total / wall / 1e9 / HBM_PEAK_GBS}}


def ms_tc_bench(steps, N=150, tol=1e-6):
    """The paper's example test: the basic scheme on a synthetic
    metal-matrix composite (fibres 10.2 %, aspect 15) with the paper's
    phase parameters, uniaxial tension-compression under mixed boundary
    conditions (eps_xx prescribed, all other mean stresses zero), the
    reference stiffness fixed or adjusted to the tangent field every step."""
    import torch
    from paper_2006_04391_amd import api, inputs
    phase_np = inputs.mmc_phase(N, seed=4)
    phase = torch.from_numpy(phase_np).cuda()
    n = N ** 3
    h, path = inputs.tension_compression_path(steps)
    out = {"workload": f"Moulinec-Suquet basic scheme, {N}^3 synthetic metal-matrix composite "
                       f"(fibres {phase_np.mean() * 100:.1f} %, aspect 15, r = 2.5), paper's "
                       f"parameters, uniaxial tension-compression 0 -> 3.58454e-3 -> -3.48441e-3 "
                       f"at 1.4e-3/s, mixed conditions, {steps} steps of h = {h:.5f} s, tol {tol}"}
    for upd in (True, False):
        ms = api.MS((N, N, N), inputs.paper_phases(), tol=tol, max_iter=5000, ref_update=upd)
        eps = torch.zeros((6, n), dtype=torch.float64, device="cuda")
        a = torch.zeros_like(eps)
        ms.step_mixed(phase, [0.0] * 6, h, eps, a, 0b111110)   # warm-up (plans, modules)
        eps.zero_()
        a.zero_()
        ms.set_macro([0.0] * 6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, curve, fails = [], [], 0
        for e in path:
            mean, Er, it, _ = ms.step_mixed(phase, [e, 0, 0, 0, 0, 0], h, eps, a, 0b111110)
            iters.append(it)
            curve.append((e, mean[0]))
            fails += ms.newton_failures()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms.close()
        total = sum(iters)
        key = "reference_update" if upd else "reference_fixed"
        out[key] = {"wall_s": wall, "iterations_total": total, "iterations": iters,
                    "point_solves_not_converged": fails,
                    "ms_per_iteration": wall / total * 1e3,
                    "sweep_updates_per_s": total * n / wall,
                    "stress_strain": curve[:: max(1, steps // 16)] + [curve[-1]]}
        log(f"[bench] MS tension-compression {N}^3 ({key}): {steps} steps, {total} iterations, "
            f"{wall:.2f} s, {wall / total * 1e3:.3f} ms/iteration, {fails} point solves not converged")
        del eps, a
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--side", type=int, default=256, help="cube side (256 = the headline batch)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tangent", action="store_true", help="skip the tangent variant")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests in the serving stream (0 skips the serving leg)")
    ap.add_argument("--serve-cap", type=int, default=1 << 24,
                    help="points per batched launch (latency-aware batch shaping; 0 = unbounded)")
    ap.add_argument("--serve-workers", type=int, default=8,
                    help="host processes generating the requests' microstructures")
    ap.add_argument("--ms-steps", type=int, default=20,
                    help="load steps of the 128^3 Moulinec-Suquet run (0 skips it)")
    ap.add_argument("--tc-steps", type=int, default=80,
                    help="load steps of the 150^3 tension-compression test (0 skips it)")
    ap.add_argument("--no-rk23", action="store_true", help="skip the adaptive ode23 and ode12 legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (known traffic: 1 GiB read, "
                         "1 GiB written) so profiler byte counters can be scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not "
                                   "supported (the per-point path would shard by contiguous "
                                   "point ranges, one range per GPU)"}))
        sys.exit(2)

    # the serving stream's microstructures are generated in worker processes
    # before the GPU is initialised
    serve_reqs = serve_fields = None
    if args.serve_requests > 0:
        from paper_2006_04391_amd import inputs, serve
        t0 = time.perf_counter()
        serve_reqs = inputs.serving_requests(count=args.serve_requests, rate=200.0, seed=4)
        serve_fields = serve.prepare_fields(serve_reqs, workers=args.serve_workers)
        log(f"[bench] serving stream: {len(serve_reqs)} requests, "
            f"{sum(q.n for q in serve_reqs):.3e} voxels, generated in "
            f"{time.perf_counter() - t0:.1f} s")

    import torch
    from paper_2006_04391_amd import api, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    ps = inputs.points_c1(N=args.side) if args.side != 256 else inputs.points_c1()
    log(f"[bench] inputs {ps.n} points generated in {time.perf_counter() - t0:.1f} s")
    n = ps.n
    eps = torch.from_numpy(ps.eps).to(dev)
    a_old = torch.from_numpy(ps.a_old).to(dev)
    phase = torch.from_numpy(ps.phase).to(dev)
    sigma = torch.empty_like(eps)
    a_new = torch.empty_like(a_old)
    stream = torch.cuda.current_stream(dev)

    def step():
        api.evaluate(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                     sigma_out=sigma, a_out=a_new)

    total_ms, each, wall = time_calls(step, args.steps, args.warmup, stream)
    ms = total_ms / args.steps
    value = n / (ms * 1e-3)
    # the roofline figures use the same time as ms_per_step
    achieved = BYTES_PER_POINT * n / (ms * 1e-3) / 1e9
    log(f"[bench] forward: {ms:.3f} ms/step, {value:.3e} updates/s, {achieved:.0f} GB/s "
        f"(per-launch events: median {np.median(each):.3f} ms)")

    # iteration profile of the batch (for the FLOP side of the roofline)
    _, _, iters, cnt = api.evaluate(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                                    return_iters=True)
    it = iters.cpu().numpy()
    hist = {int(k): int(v) for k, v in zip(*np.unique(it, return_counts=True))}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.side}^3 periodic fibre composite (15 % fibres r=4 L=64), one "
                        "implicit-Euler evaluation batch without tangent, h=0.1 s, tol 1e-12",
            "points": n,
            "newton_updates_histogram": hist,
            "nonconverged": int(cnt.item()),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": MEASURED_TRAFFIC.get(kernel_source_hash()),
            "kernel": "gsm_eval_kernel<MSGSM, false, false>",
            "kernel_source_hash": kernel_source_hash(),
            "bytes_per_point": BYTES_PER_POINT,
        },
    }
    out["launch_ms_median"] = float(np.median(each))
    fpp = MEASURED_FP64_FLOP_PER_POINT.get(kernel_source_hash())
    if fpp is not None:
        tf = fpp * n / (ms * 1e-3) / 1e12
        out["roofline"]["fp64"] = {"executed_flop_per_point": fpp, "achieved": tf,
                                   "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": tf / FP64_PEAK_TFLOPS}

    # the same batch with a non-integer power-law exponent (n = 5.1): every
    # exponent takes the same exp/log path, so this costs what n = 5 costs
    ph51 = [dict(ps.phases[0], n=5.1), ps.phases[1]]

    def step51():
        api.evaluate(eps, a_old, phase, ph51, ps.h, ps.tol, ps.max_iter,
                     sigma_out=sigma, a_out=a_new)
    t51, _, _ = time_calls(step51, args.steps, args.warmup, stream)
    ms51 = t51 / args.steps
    a51 = BYTES_PER_POINT * n / (ms51 * 1e-3) / 1e9
    out["exponent_5_1"] = {"workload": "same 256^3 batch, matrix exponent n = 5.1",
                           "ms_per_step": ms51, "value": n / (ms51 * 1e-3), "unit": "updates/s",
                           "roofline_frac": a51 / HBM_PEAK_GBS,
                           "roofline": hbm_roofline(BYTES_PER_POINT, n, ms51)}
    log(f"[bench] n = 5.1: {ms51:.3f} ms/step, {a51 / HBM_PEAK_GBS:.3f} of the HBM roofline")

    out["latency_4096"] = latency_c0(dev)

    if not args.no_tangent:
        # the tangent field (36 doubles per point, 4.8 GB) is allocated once,
        # outside the timed region
        tan_out = torch.empty((36, n), dtype=torch.float64, device=dev)

        def step_t():
            api.evaluate(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                         sigma_out=sigma, a_out=a_new, tangent=True, tangent_out=tan_out)
        tt, each_t, _ = time_calls(step_t, max(5, args.steps // 2), 2, stream)
        ms_t = tt / max(5, args.steps // 2)
        out["tangent"] = {"ms_per_step": ms_t, "value": n / (ms_t * 1e-3), "unit": "updates/s",
                          "hbm_gbs": BYTES_PER_POINT_TANGENT * n / (ms_t * 1e-3) / 1e9,
                          "roofline": hbm_roofline(BYTES_PER_POINT_TANGENT, n, ms_t)}
        log(f"[bench] tangent: {ms_t:.3f} ms/step")

    # the paper's conventional strategy (hand-reduced radial return, no AD)
    # on the same batch: what the automatic evaluation costs
    def step_cv():
        api.evaluate_conventional(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                                  sigma_out=sigma, a_out=a_new)
    tc, _, _ = time_calls(step_cv, max(3, args.steps // 2), 2, stream)
    ms_cv = tc / max(3, args.steps // 2)
    out["conventional"] = {"workload": "same 256^3 batch, radial return (scalar Newton, no AD)",
                           "ms_per_step": ms_cv, "value": n / (ms_cv * 1e-3), "unit": "updates/s",
                           "automatic_over_conventional_time": ms / ms_cv,
                           "roofline": hbm_roofline(BYTES_PER_POINT_CONVENTIONAL, n, ms_cv)}
    log(f"[bench] conventional: {ms_cv:.3f} ms/step (automatic / conventional = {ms / ms_cv:.2f})")
    if not args.no_tangent:
        def step_cvt():
            api.evaluate_conventional(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                                      sigma_out=sigma, a_out=a_new, tangent=True,
                                      tangent_out=tan_out)
        tct, _, _ = time_calls(step_cvt, max(5, args.steps // 2), 2, stream)
        cv_t = tct / max(5, args.steps // 2)
        out["conventional"]["tangent_ms_per_step"] = cv_t
        out["conventional"]["tangent_roofline"] = hbm_roofline(
            BYTES_PER_POINT_CONVENTIONAL + 36 * 8, n, cv_t)
        if "tangent" in out:
            out["conventional"]["automatic_over_conventional_time_tangent"] = (
                out["tangent"]["ms_per_step"] / cv_t)
        log(f"[bench] conventional with tangent: {cv_t:.3f} ms/step")

    # the paper's semi-automatic strategy: the same Newton solve and tangent
    # with hand-derived partials of omega and Psi instead of AD
    from paper_2006_04391_amd import _lib as _l

    def step_sa():
        api.evaluate(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                     sigma_out=sigma, a_out=a_new, flags=_l.HAND_PARTIALS)
    ts, _, _ = time_calls(step_sa, max(3, args.steps // 2), 2, stream)
    ms_sa = ts / max(3, args.steps // 2)
    sa = {"workload": "same 256^3 batch, hand-derived partials in the generic Newton solve",
          "ms_per_step": ms_sa, "value": n / (ms_sa * 1e-3), "unit": "updates/s",
          "automatic_over_semi_automatic_time": ms / ms_sa,
          "roofline": hbm_roofline(BYTES_PER_POINT, n, ms_sa)}
    if not args.no_tangent:
        def step_sat():
            api.evaluate(eps, a_old, phase, ps.phases, ps.h, ps.tol, ps.max_iter,
                         sigma_out=sigma, a_out=a_new, tangent=True, flags=_l.HAND_PARTIALS,
                         tangent_out=tan_out)
        tst, _, _ = time_calls(step_sat, max(5, args.steps // 2), 2, stream)
        sa["tangent_ms_per_step"] = tst / max(5, args.steps // 2)
        sa["tangent_roofline"] = hbm_roofline(BYTES_PER_POINT_TANGENT, n,
                                              sa["tangent_ms_per_step"])
        if "tangent" in out:
            sa["automatic_over_semi_automatic_time_tangent"] = (out["tangent"]["ms_per_step"] /
                                                                sa["tangent_ms_per_step"])
    out["semi_automatic"] = sa

    log(f"[bench] semi-automatic: {ms_sa:.3f} ms/step (automatic / semi-automatic = "
        f"{ms / ms_sa:.2f})" + (f", tangent {sa['tangent_ms_per_step']:.3f} ms/step"
                               if "tangent_ms_per_step" in sa else ""))

    # single precision (float fields and arithmetic, hand-derived partials)
    eps32 = eps.float()
    a32 = a_old.float()
    sig32 = torch.empty_like(eps32)
    an32 = torch.empty_like(a32)

    def step_32():
        api.evaluate_f32(eps32, a32, phase, ps.phases, ps.h, 1e-6, ps.max_iter,
                         sigma_out=sig32, a_out=an32)
    t32, _, _ = time_calls(step_32, max(3, args.steps // 2), 2, stream)
    ms_32 = t32 / max(3, args.steps // 2)
    f32 = {"workload": "same 256^3 batch rounded to float32, FP32 arithmetic, tol 1e-6 (floor "
                       "at the FP32 rounding level)",
           "ms_per_step": ms_32, "value": n / (ms_32 * 1e-3), "unit": "updates/s",
           "bytes_per_point": BYTES_PER_POINT_F32,
           "hbm_gbs": BYTES_PER_POINT_F32 * n / (ms_32 * 1e-3) / 1e9,
           "fp64_over_fp32_time": ms / ms_32,
           "roofline": hbm_roofline(BYTES_PER_POINT_F32, n, ms_32)}
    if not args.no_tangent:
        tan32 = torch.empty((36, n), dtype=torch.float32, device=dev)

        def step_32t():
            api.evaluate_f32(eps32, a32, phase, ps.phases, ps.h, 1e-6, ps.max_iter,
                             sigma_out=sig32, a_out=an32, tangent=True, tangent_out=tan32)
        t32t, _, _ = time_calls(step_32t, max(5, args.steps // 2), 2, stream)
        f32["tangent_ms_per_step"] = t32t / max(5, args.steps // 2)
        f32["tangent_roofline"] = hbm_roofline(BYTES_PER_POINT_F32_TANGENT, n,
                                               f32["tangent_ms_per_step"])
        del tan32
        if "tangent" in out:
            f32["fp64_over_fp32_time_tangent"] = (out["tangent"]["ms_per_step"] /
                                                  f32["tangent_ms_per_step"])
    out["fp32"] = f32
    log(f"[bench] fp32: {ms_32:.3f} ms/step (fp64 / fp32 = {ms / ms_32:.2f})" +
        (f", tangent {f32['tangent_ms_per_step']:.3f} ms/step" if "tangent_ms_per_step" in f32
         else ""))
    del eps32, a32, sig32, an32

    if not args.no_rk23:
        # adaptive explicit Runge-Kutta over one load step of the same batch:
        # the strain ramps from 0.8 eps to eps (the last step of a 5-step path)
        eps_n = 0.8 * eps
        a_rk = torch.empty_like(a_old)
        tan_rk = None
        for pair, fn in (("rk23", api.evaluate_rk23), ("rk12", api.evaluate_rk12)):
            steps_rk = {}

            def step_rk():
                s_, _, st, _ = fn(eps_n, eps, a_old, phase, ps.phases, h=ps.h,
                                  sigma_out=sigma, a_out=a_rk)
                steps_rk["last"] = st
            tr, _, _ = time_calls(step_rk, max(3, args.steps // 4), 1, stream)
            ms_rk = tr / max(3, args.steps // 4)
            st = steps_rk["last"].cpu().numpy()
            name = "Bogacki-Shampine 3(2)" if pair == "rk23" else "Heun-Euler 2(1)"
            out[pair] = {"workload": f"same 256^3 batch, {name}, strain ramp 0.8 eps -> eps over "
                                     "h = 0.1 s, atol 1e-6, rtol 1e-3 (no tangent)",
                         "ms_per_step": ms_rk, "value": n / (ms_rk * 1e-3), "unit": "updates/s",
                         "accepted_steps_histogram": {int(k): int(v) for k, v in
                                                      zip(*np.unique(st, return_counts=True))},
                         "roofline": hbm_roofline(BYTES_PER_POINT_RK, n, ms_rk)}
            log(f"[bench] {pair}: {ms_rk:.3f} ms/step")
            # with the consistent tangent (the sensitivity system integrated
            # alongside and inside the error measure)
            if tan_rk is None:
                tan_rk = torch.empty((36, n), dtype=torch.float64, device=dev)

            def step_rk_t():
                r = fn(eps_n, eps, a_old, phase, ps.phases, h=ps.h, tangent=True,
                       sigma_out=sigma, a_out=a_rk, tangent_out=tan_rk)
                steps_rk["tan"] = r[3]
            tt_rk, _, _ = time_calls(step_rk_t, 3, 1, stream)
            ms_rk_t = tt_rk / 3
            st_t = steps_rk["tan"].cpu().numpy()
            out[pair]["tangent_ms_per_step"] = ms_rk_t
            # bound by the FP64 work of its stage Hessians and sensitivity
            # columns, not by memory: the HBM fraction shows how far
            out[pair]["tangent_roofline"] = hbm_roofline(BYTES_PER_POINT_RK_TANGENT, n, ms_rk_t)
            out[pair]["tangent_accepted_steps_histogram"] = {
                int(k): int(v) for k, v in zip(*np.unique(st_t, return_counts=True))}
            log(f"[bench] {pair} with tangent: {ms_rk_t:.3f} ms/step")
        del eps_n, a_rk, tan_rk

    if args.ms_steps > 0:
        out["ms"] = ms_bench(args.ms_steps)
    if args.tc_steps > 0:
        out["ms_tension_compression"] = ms_tc_bench(args.tc_steps)

    if serve_reqs is not None:
        from paper_2006_04391_amd import serve
        del eps, a_old, phase, sigma, a_new
        torch.cuda.empty_cache()
        sv = {"workload": f"{len(serve_reqs)} requests, Poisson arrivals 200/s, cube side "
                          "log-uniform in [32, 256], fibre or sphere microstructure, phase "
                          "parameters jittered +-10 %, 1-10 load steps each, HBM budget 200 GB; "
                          f"batched launches capped at {args.serve_cap} points (four times that "
                          "while requests wait in the queue), least remaining work first"}
        for saturate in (False, True):
            for sequential in (False, True):
                r = serve.replay(serve_reqs, serve_fields, sequential=sequential,
                                 saturate=saturate,
                                 max_batch_points=0 if sequential else args.serve_cap)
                key = ("saturated_" if saturate else "poisson_") + r["mode"]
                sv[key] = r
                log(f"[bench] serving {key}: {r['throughput']:.3e} updates/s, "
                    f"p50 {r['latency_p50_s'] * 1e3:.1f} ms, p99 {r['latency_p99_s'] * 1e3:.1f} ms, "
                    f"{r['launches']} launches, makespan {r['makespan_s']:.2f} s")
        out["serving"] = sv
        del serve_fields

    if not args.no_cpu:
        log("[bench] timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(ps)
        log(f"[bench] cpu baseline {out['cpu_baseline']}")

    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
        # the rate of a plain device copy: what the memory system gives a
        # kernel that only streams (read + write bytes over the time)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(10):
            dst.copy_(src)
        c1.record()
        torch.cuda.synchronize()
        out["copy_gbs"] = 2 * src.numel() * 8 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        log(f"[bench] 1 GiB device copy: {out['copy_gbs']:.0f} GB/s (read + write)")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
