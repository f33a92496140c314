"""Benchmark of the HEOM RK4 hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision P]

One step is one classic RK4 step (four right-hand-side evaluations over every
ADO, fused into four stage launches).  The default workload is the 48-site
aggregate (W = 96 modes, depth 3, 156849 ADOs of 48x48, FP32 bulk with FP64
sigma_0 and observables), the largest configuration and the one whose working
set (about 15 GB) is bound by HBM bandwidth.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import heom_inputs as hi  # noqa: E402

METRIC = "HEOM ADO-updates/s + HBM GB/s; serve p50/p99 latency vs plain FP64"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "aggregate48": lambda: hi.aggregate48(),
    "aggregate24": lambda: hi.aggregate24(),
    "fmo_like": lambda: hi.fmo_like(),
    "dimer": lambda: hi.dimer(),
    # the largest request of the serving mix as a single propagation
    # (14 sites, W = 28, depth 5: 237336 ADOs of 14x14, FMA kernel)
    "mix_largest": lambda: _mix_largest(),
    # the paper's FMO reference setting (D, K) = (6, 6) with the Pade
    # expansion at 300 K: 7 sites, 5 poles per bath, 12271512 ADOs of 7x7;
    # dt = 0.1 fs (the step-size guard's limit for these rates is 0.14 fs)
    "fmo66_pade": lambda: hi.fmo_like_pade(300.0, 6, 5, n_steps=20, dt_fs=0.1),
}


def _mix_largest():
    from math import comb
    reqs = hi.serving_mix(n_requests=128, seed=512, n_steps=200)
    def size(r):
        W = sum(b["matsubara"] + 1 for b in r["runs"][0]["baths"])
        return comb(W + r["depth"], W) * r["N"] ** 2
    run = dict(max(reqs, key=size)["runs"][0])
    run["record_every"] = 10
    return run


# the device sources that define each stage kernel (its own file and the
# shared helpers and launchers)
KERNEL_SOURCES = {
    "k_stage_persist": ("heom_kernels.hip", "heom_stage_persist.inc"),
    "k_stage_small": ("heom_kernels.hip", "heom_stage_small.inc"),
}


def _kernel_source_digest(kernel):
    """SHA-256 over the device sources of `kernel`, in the order listed."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(kernel, ("heom_kernels.hip",)):
        with open(os.path.join(ROOT, "paper_1803_03498_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when there is none or
    the kernel source has changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.txt" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != _kernel_source_digest(kernel):
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="aggregate48",
                    choices=sorted(WORKLOADS) + ["serve", "copy", "fluorescence", "absorption"])
    ap.add_argument("--copy-gib", type=float, default=4.0,
                    help="--workload copy: bytes read (and written) per copy")
    ap.add_argument("--precision", default="fp32_mixed", choices=["fp32_mixed", "fp32_herm", "fp64"])
    ap.add_argument("--cpu-baseline-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample (0 disables it)")
    ap.add_argument("--no-fp64-check", action="store_true",
                    help="skip the untimed FP64 run of the same steps")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests in the serving mix (a prefix is run, see --serve-seconds)")
    ap.add_argument("--serve-steps", type=int, default=1000)
    ap.add_argument("--serve-seconds", type=float, default=150.0,
                    help="time the serving replays may take (0 skips the serving leg)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-arena-gb", type=float, default=48.0)
    ap.add_argument("--serve-cpu-requests", type=int, default=128,
                    help="requests of the mix timed on the oracle (the first ones)")
    ap.add_argument("--serve-log", default=None,
                    help="write one JSON line per served request to this file")
    return ap.parse_args()


def cpu_baseline(prob, target_s):
    """Time the FP64 oracle on a bounded sample of the same workload,
    single-threaded on this host: the oracle's own RK4 step code (four
    evaluations and the vector updates) over every k-th ADO of the
    hierarchy, all levels, with the model built outside the timed region
    (oracle.time_step_sample); k is set from a first probe so that the
    sample takes about target_s.  One ADO-update is one ADO advanced by one
    RK4 step."""
    import oracle
    _, n = oracle.sizes(prob)
    N = prob["H"].shape[0]
    x = np.zeros((n, N, N), np.complex128)  # pages are touched only where read
    x[0] = prob["rho0"]
    t0 = time.perf_counter()
    oracle.rhs(prob, x, 0, 0)  # model and table construction only
    t_setup = time.perf_counter() - t0
    stride = max(1, n // 256)
    sec = oracle.time_step_sample(prob, x, prob["dt_fs"], 0, n, stride, 1)
    per_ado = max(sec, 1e-9) / ((n + stride - 1) // stride)
    stride = max(1, min(stride, int(n * per_ado / target_s)))
    # a step shorter than the target is repeated (the fastest repetition)
    reps = 1 if stride > 1 else max(1, min(100, int(target_s / max(per_ado * n, 1e-9))))
    sec = oracle.time_step_sample(prob, x, prob["dt_fs"], 0, n, stride, reps)
    k = (n + stride - 1) // stride
    which = ("every ADO" if stride == 1 else "every %d-th ADO" % stride)
    return {"value": k / max(sec, 1e-9), "unit": "ADO-updates/s", "cores": 1,
            "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "threads_available": len(os.sched_getaffinity(0)),
            "sample": "FP64 oracle RK4 step (four right-hand sides and the vector updates) "
                      "over %s of %s (%d of %d, all levels), %.2f s of CPU on one thread%s; "
                      "model setup (%.1f s per build) outside the timed region"
                      % (which, prob.get("name", "?"), k, n, sec,
                         ", fastest of %d repetitions" % reps if reps > 1 else "", t_setup)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _bulk_kernel_name(info, precision, N, heom):
    """The stage kernel that propagates ADOs u >= 1 of a Hermitian run."""
    if precision == heom.FP32_MIXED and 10 <= N <= 64:
        return "k_stage_persist"
    if not info["bulk_kernel"]:
        # single propagations with N <= 16 and >= 32768 ADOs take the
        # persistent FMA kernel
        return "k_stage_small" if N <= 16 and info["n_ado"] >= 32768 else "k_bulk_fma"
    return "k_bulk_mfma_pk" if precision == heom.FP32_HERM else "k_bulk_mfma"


def _table_bytes_per_launch(kernel, n, W, D, fp64):
    """Bytes of link tables and coefficients that one stage launch reads for
    the ADOs u >= 1, outside the algorithmic bytes: per ADO its "-" links
    (neighbour and mode, state, the two weights) and its damping rate, and
    per ADO below the top level its "+" links (neighbour, weight); the
    FP64-coefficient kernels read the weights in FP64, the level-major FP64
    matrix-core kernel also the level byte."""
    from math import comb
    Dm = max(D, 1)
    n_low = comb(W + D - 1, W) - 1 if D >= 1 and W >= 1 else 0
    w_bytes = 16 if fp64 else 8
    per_ado = Dm * (8 + 4 + w_bytes) + 8 + (1 if kernel == "k_bulk_mfma" else 0)
    return float((n - 1) * per_ado + n_low * W * (4 + 8))


def _fp64_reference(heom, torch, lib, prob, precision, steps, rec_every, N, n):
    """The benchmarked steps from the initial state in FP64 (timed, with its
    bulk-kernel events) and in `precision`; returns the FP64 figures and the
    largest population difference over the records."""
    out = {}
    recs = {}
    for prec in (heom.FP64, precision):
        h = heom.Hierarchy(prob, prec)
        st = h.new_state(prob["rho0"])
        work = h.workspace(steps, rec_every, heom.OBS_POPULATION)
        torch.cuda.synchronize()
        if prec == heom.FP64:
            lib.heom_timing_enable(1)
            lib.heom_timing_read(None, None, None, 1)
        t0 = time.perf_counter()
        recs[prec] = h.propagate(st, prob["dt_fs"], steps, rec_every, hermitian=True, work=work)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if prec == heom.FP64:
            lib.heom_timing_enable(0)
            ms = ctypes.c_double()
            launches = ctypes.c_int64()
            kbytes = ctypes.c_double()
            lib.heom_timing_read(ctypes.byref(ms), ctypes.byref(launches), ctypes.byref(kbytes), 1)
            avg = ms.value / 1e3 / max(launches.value, 1)
            achieved = kbytes.value / max(launches.value, 1) / avg / 1e9
            out.update({"ms_per_step": 1e3 * el / steps, "ado_updates_per_s": n * steps / el,
                        "bulk_kernel": _bulk_kernel_name(h.info, prec, N, heom),
                        "avg_launch_ms": avg * 1e3, "achieved_GBps": achieved,
                        "frac": achieved / HBM_PEAK_GBS, "steps": steps,
                        "note": "complex128 throughout, same workload, untimed in the line's value"})
        del st, work, h
        torch.cuda.empty_cache()
    a, b = recs[heom.FP64], recs[precision]
    out["fp32_vs_fp64_max_population_error"] = float(np.max(np.abs(a[:, :N] - b[:, :N])))
    out["fp32_trace_drift"] = float(np.max(np.abs(b[:, N] - 1.0)))
    # max |sigma_0 - sigma_0^+| over the records (column N + 2 of a
    # population record)
    out["fp32_hermiticity_residual"] = float(np.max(b[:, N + 2]))
    out["fp64_hermiticity_residual"] = float(np.max(a[:, N + 2]))
    out["fp64_trace_drift"] = float(np.max(np.abs(a[:, N] - 1.0)))
    out["records_compared"] = int(a.shape[0])
    return out


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def _replay(heom, reqs, precision, max_active, arena_bytes, rate, form=0, timeout_s=900.0,
            log=None, tag="", keep=None):
    """Submit requests at their (scaled) Poisson arrival times (all at once
    when rate is None); returns per-request latencies (s), the makespan (s),
    the ADO-updates done, the number of requests run in the coherence-block
    form and each request's service time (finish - admission, s).  keep: a
    dict that receives each request's records by request id."""
    srv = heom.Server(arena_bytes, max_active)
    t0 = time.monotonic()
    arrival = 0.0
    tickets = []
    for k, r in enumerate(reqs):
        if rate is not None:
            arrival += r["gap"] / rate
            delay = t0 + arrival - time.monotonic()
            if delay > 0:
                time.sleep(delay)
        tickets.append(srv.submit(r["runs"], precision, form=form))
    lat, work, n_block, service = [], 0, 0, []
    t_end = t0
    for k, (r, t) in enumerate(zip(reqs, tickets)):
        res = srv.wait(t, timeout_s)
        if res["status"] != 0:
            raise RuntimeError("request %d failed: %s" % (r["id"], res["status"]))
        lat.append(res["t_finish"] - res["t_submit"])
        service.append(res["t_finish"] - res["t_admit"])
        t_end = max(t_end, res["t_finish"])
        ado_updates = r["n_ado"] * r["runs"][0]["n_steps"] * len(r["runs"])
        work += ado_updates
        n_block += res["form"] == 2
        if keep is not None:
            keep[r["id"]] = res["records"]
        if log is not None:
            log.write(json.dumps({
                "replay": tag, "request": r["id"], "kind": r["kind"], "N": r["N"],
                "depth": r["depth"], "matsubara": r["matsubara"], "n_ado": r["n_ado"],
                "runs": len(r["runs"]), "form": "block" if res["form"] == 2 else "full",
                "queue_ms": 1e3 * (res["t_admit"] - res["t_submit"]),
                "latency_ms": 1e3 * (res["t_finish"] - res["t_submit"]),
                "ado_updates": ado_updates}) + "\n")
        srv.release(t)
    srv.close()
    if log is not None:
        log.flush()
    # t_finish is on the library's monotonic clock, like time.monotonic here
    return lat, max(t_end - t0, 1e-9), work, n_block, service


def _full_bytes(r):
    """Bytes of one RK4 stage copy of a request on full matrices."""
    return r["n_ado"] * r["N_full"] ** 2 * len(r["runs"])


def _serve_stats(lat, span, work, n):
    return {"p50_ms": 1e3 * _percentile(lat, 50), "p99_ms": 1e3 * _percentile(lat, 99),
            "throughput_req_per_s": n / span, "ado_updates_per_s": work / span,
            "makespan_s": span}


def _oracle_request_seconds(task):
    """CPU seconds of the FP64 oracle for one whole request on this core:
    per run, its model setup plus n_steps RK4 steps (the runs of a request
    differ only in their initial state and dipole).  The step is the
    oracle's own step code timed on every stride-th ADO (all of them when
    that fits `budget`), scaled to all ADOs; the smaller of two timings.
    Returns (seconds, stride)."""
    runs, n_steps, budget = task
    import oracle
    p = runs[0]
    N = np.asarray(p["H"]).shape[0]
    _, n = oracle.sizes(p)
    x = np.zeros((n, N, N), np.complex128)  # pages are touched only where read
    x[0] = p["rho0"]
    t_setup = float("inf")
    for _ in range(2):  # model and table construction only (each call builds them)
        t0 = time.perf_counter()
        oracle.rhs(p, x, 0, 0)
        t_setup = min(t_setup, time.perf_counter() - t0)
    stride = max(1, n // 256)
    while True:
        sec = oracle.time_step_sample(p, x, p["dt_fs"], 0, n, stride, 2)
        if stride == 1 or sec > 0.1 * budget:
            break
        stride = max(1, stride // 8)
    step = sec * stride * n / (n + stride - 1 - (n - 1) % stride)  # per sampled ADO x n
    return len(runs) * (t_setup + step * n_steps), stride


def serve_cpu_oracle(mix, n_steps, target_s):
    """The FP64 oracle on every host core as independent processes, one
    request at a time each, over the whole mix: each request's CPU time is
    measured on a bounded sample (see _oracle_request_seconds) while all
    processes run, so memory contention is included.  Runs before the GPU is
    touched (its worker processes are spawned)."""
    import multiprocessing as mp
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    budget = min(3.0, max(0.05, target_s * procs / max(len(mix), 1)))
    # largest first (an ADO costs about N^3), so that the longest single
    # steps do not come last
    cost = [r["n_ado_est"] * r["N"] ** 3 for r in mix]
    order = sorted(range(len(mix)), key=lambda i: -cost[i])
    tasks = [(mix[i]["runs"], n_steps, budget) for i in order]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_request_seconds, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    secs, steps = [0.0] * len(mix), [0] * len(mix)
    for i, (sec, st) in zip(order, res):
        secs[i], steps[i] = sec, st
    return {"seconds": secs, "steps_timed": steps, "procs": procs, "budget_s": budget,
            "wall_s": wall}


def _serve_cpu_baseline(cpu, n):
    """Requests/s of the oracle on cpu["procs"] cores for the first n
    requests (each core runs whole requests one after another)."""
    n = min(n, len(cpu["seconds"]))
    secs = cpu["seconds"][:n]
    mean = sum(secs) / max(len(secs), 1)
    sampled = sum(1 for s in cpu["steps_timed"][:n] if s > 1)
    return {"value": cpu["procs"] / mean, "unit": "req/s", "cores": cpu["procs"],
            "kind": "oracle", "cpu_model": _cpu_model(),
            "p50_request_s_one_core": _percentile(secs, 50),
            "p99_request_s_one_core": _percentile(secs, 99),
            "sample": "FP64 oracle on %d host cores as independent processes, one request each "
                      "at a time, over the first %d requests of the mix: each request's RK4 "
                      "step timed with the oracle's step code over all its ADOs (%d requests) "
                      "or every k-th ADO (%d, k chosen so the sample takes about %.2f s) and "
                      "scaled to all ADOs, its steps and runs, plus its model setup per run; "
                      "%.0f s wall for the sample"
                      % (cpu["procs"], n, n - sampled, sampled, 0.1 * cpu["budget_s"],
                         cpu["wall_s"])}


def _serve_accuracy(heom, reqs, got, ref):
    """Errors of the batched FP32-mixed results against the plain FP64 ones
    (the FP64 path, itself held to the oracle at 1e-12 by the parity
    tests) over the same requests: population error, trace drift and
    Hermiticity residual of the population requests, and for the absorption
    requests the dipole-response error and the spectrum error (trapezoid DFT
    over 1 ps on the -1000..1000 cm^-1 grid, max |S - S_ref| / max |S_ref|)."""
    w = np.arange(-1000.0, 1001.0, 1.0)
    out = {"requests_compared": 0, "population_requests": 0, "absorption_requests": 0,
           "max_population_error": 0.0, "max_trace_drift": 0.0,
           "max_hermiticity_residual": 0.0, "max_dipole_response_error": 0.0,
           "max_spectrum_rel_error": 0.0}
    for r in reqs:
        a, b = got.get(r["id"]), ref.get(r["id"])
        if a is None or b is None:
            continue
        out["requests_compared"] += 1
        dt = r["runs"][0]["dt_fs"] * r["runs"][0]["record_every"]
        if r["kind"] == "population":
            N = np.asarray(r["runs"][0]["H"]).shape[0]
            out["population_requests"] += 1
            out["max_population_error"] = max(out["max_population_error"],
                                               float(np.max(np.abs(a[..., :N] - b[..., :N]))))
            out["max_trace_drift"] = max(out["max_trace_drift"],
                                         float(np.max(np.abs(a[..., N] - 1.0))))
            out["max_hermiticity_residual"] = max(out["max_hermiticity_residual"],
                                                  float(np.max(a[..., N + 2])))
        else:
            out["absorption_requests"] += 1
            Pa = a[:, :, 0] + 1j * a[:, :, 1]
            Pb = b[:, :, 0] + 1j * b[:, :, 1]
            out["max_dipole_response_error"] = max(out["max_dipole_response_error"],
                                                   float(np.max(np.abs(Pa - Pb))))
            Sa, Sb = heom.spectrum(Pa, dt, w), heom.spectrum(Pb, dt, w)
            out["max_spectrum_rel_error"] = max(
                out["max_spectrum_rel_error"],
                float(np.max(np.abs(Sa - Sb)) / max(np.max(np.abs(Sb)), 1e-300)))
    return out


def serve_leg(args, cpu=None):
    """Serving mix (seed 512): continuous batching in FP32-mixed, with the
    coherence-block form for absorption requests, against plain FP64
    one-solve-at-a-time on full matrices, on the same Poisson traces at
    0.5x, 0.8x and 1.0x of the batched server's closed-loop capacity.  The
    longest prefix of the mix whose replays fit --serve-seconds is run."""
    import torch

    import paper_1803_03498_amd as heom
    torch.cuda.set_device(0)
    mix = hi.serving_mix(n_requests=args.serve_requests, seed=512, n_steps=args.serve_steps)
    for r in mix:
        r["n_ado"] = heom.plan(r["runs"][0])["n_ado"]
        r["N_full"] = np.asarray(r["runs"][0]["H"]).shape[0]
    arena = int(args.serve_arena_gb * (1 << 30))
    slots = args.serve_slots
    loads = (0.5, 0.8, 1.0)
    log = open(args.serve_log, "w") if args.serve_log else None
    print("serve: warm-up and pilot", file=sys.stderr, flush=True)
    _replay(heom, mix[:4], heom.FP32_MIXED, 8, arena, None)
    _replay(heom, mix[:2], heom.FP64, 1, arena, None, form=1)
    torch.cuda.synchronize()
    # pilot on the first requests (closed loop): the batched server's time per
    # full-matrix byte, and plain FP64 service times fitted as a + b * bytes
    n_pilot = min(32, len(mix))
    pilot = mix[:n_pilot]
    _, span_pb, _, _, _ = _replay(heom, pilot, heom.FP32_MIXED, slots, arena, None)
    _, _, _, _, svc = _replay(heom, pilot[:16], heom.FP64, 1, arena, None, form=1)
    x = np.array([_full_bytes(r) for r in pilot[:16]], float)
    A = np.stack([np.ones_like(x), x], 1)
    a, b = np.linalg.lstsq(A, np.array(svc), rcond=None)[0]
    a, b = max(a, 0.0), max(b, 0.0)
    b_per_byte = span_pb / sum(_full_bytes(r) for r in pilot)

    def estimate(k):
        wb = sum(_full_bytes(r) for r in mix[:k])
        tb, tf = b_per_byte * wb, a * k + b * wb
        # closed loop + three batched replays + three plain FP64 replays (each
        # service-bound once the arrivals outpace plain FP64)
        return tb * (1.0 + sum(1.0 / y for y in loads)) + sum(max(tf, tb / y) for y in loads)

    n = len(mix)
    while n > 16 and estimate(n) > args.serve_seconds:
        n -= 8
    reqs = mix[:n]
    print("serve: pilot: batched %.3g s per 1e9 elements, plain FP64 %.3f s + %.3g s per 1e9 elements per request: %d of "
          "%d requests, estimated %.0f s" % (b_per_byte * 1e9, a, b * 1e9, n, len(mix),
                                             estimate(n)), file=sys.stderr, flush=True)
    lat_c, span_c, work_c, n_block, _ = _replay(heom, reqs, heom.FP32_MIXED, slots, arena, None,
                                                log=log, tag="closed_loop")
    capacity = n / span_c
    out = {
        "requests": n, "requests_in_mix": len(mix),
        "requests_block_form": n_block,
        "steps_per_request": args.serve_steps, "slots": slots, "arena_GB": args.serve_arena_gb,
        "capacity_req_per_s": capacity,
        "closed_loop": _serve_stats(lat_c, span_c, work_c, n),
        "replays": [],
    }
    for x in loads:
        rate = x * capacity
        print("serve: replay at %.1fx capacity (%.2f req/s): batched" % (x, rate),
              file=sys.stderr, flush=True)
        # the results of the headline load are kept for their errors
        kb, kf = ({}, {}) if x == 0.8 else (None, None)
        lat_b, span_b, work_b, _, _ = _replay(heom, reqs, heom.FP32_MIXED, slots, arena, rate,
                                              log=log, tag="batched_%.1fx" % x, keep=kb)
        print("serve: replay at %.1fx capacity: plain FP64" % x, file=sys.stderr, flush=True)
        lat_f, span_f, work_f, _, _ = _replay(heom, reqs, heom.FP64, 1, arena, rate, form=1,
                                              log=log, tag="plain_fp64_%.1fx" % x, keep=kf)
        if kb is not None:
            out["accuracy_vs_fp64"] = _serve_accuracy(heom, reqs, kb, kf)
            del kb, kf
        b, f = _serve_stats(lat_b, span_b, work_b, n), _serve_stats(lat_f, span_f, work_f, n)
        out["replays"].append({
            "load": x, "arrival_rate_req_per_s": rate,
            "batched_fp32": b, "plain_fp64_one_at_a_time": f,
            "throughput_ratio": b["throughput_req_per_s"] / f["throughput_req_per_s"],
            "p99_ratio_plain_over_batched": f["p99_ms"] / b["p99_ms"]})
        print("  batched p50 %.0f p99 %.0f ms %.2f req/s | plain FP64 p50 %.0f p99 %.0f ms "
              "%.2f req/s" % (b["p50_ms"], b["p99_ms"], b["throughput_req_per_s"], f["p50_ms"],
                              f["p99_ms"], f["throughput_req_per_s"]), file=sys.stderr,
              flush=True)
    if log is not None:
        log.close()
    if cpu is not None:
        out["cpu_baseline"] = _serve_cpu_baseline(cpu, n)
    out["workload"] = ("serving mix: the first %d of %d requests (seed 512), N in 2..14, D in 2..5, "
                       "M in 0..1, population or 3-direction absorption, %d RK4 steps of 1 fs; "
                       "Poisson arrivals at 0.5x, 0.8x, 1.0x of the batched closed-loop capacity"
                       % (n, len(mix), args.serve_steps))
    return out


def _mix_cpu_oracle(args):
    """The oracle leg of the serving mix (before any GPU work), or None."""
    if args.cpu_baseline_seconds <= 0 or args.serve_seconds <= 0:
        return None
    mix = hi.serving_mix(n_requests=args.serve_requests, seed=512, n_steps=args.serve_steps)
    mix = mix[:max(1, args.serve_cpu_requests)]
    from math import comb
    for r in mix:
        W = sum(b["matsubara"] + 1 for b in r["runs"][0]["baths"])
        r["n_ado_est"] = comb(W + r["depth"], W) * len(r["runs"])
    print("serve: FP64 oracle on the host cores (%d requests)" % len(mix), file=sys.stderr,
          flush=True)
    cpu = serve_cpu_oracle(mix, args.serve_steps, args.cpu_baseline_seconds * 2)
    print("serve: oracle leg %.0f s on %d processes" % (cpu["wall_s"], cpu["procs"]),
          file=sys.stderr, flush=True)
    return cpu


def run_serve(args):
    """The serving leg on its own, as one JSON line."""
    sv = serve_leg(args, _mix_cpu_oracle(args))
    r1 = sv["replays"][-1]["batched_fp32"]
    line = {
        "metric": METRIC,
        "value": r1["ado_updates_per_s"],
        "unit": "ADO-updates/s",
        "n_gpus": 1,
        "steps": args.serve_steps,
        "warmup": 4,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sv["workload"], "slots": args.serve_slots,
                   "arena_GB": args.serve_arena_gb},
        "serve": sv,
        "roofline": None,
        "cpu_baseline": sv.get("cpu_baseline"),
    }
    print(json.dumps(line), flush=True)


def run_fluorescence(args):
    """Static fluorescence of the FMO-like system (section "Static
    Fluorescence Spectra"): thermal state by a 2 ps population run from the
    Boltzmann state, then sigma_u(inf) mu_p^+ propagated for 1 ps in each of
    three directions, and the spectrum.  Times the whole computation."""
    import torch
    import paper_1803_03498_amd as heom
    torch.cuda.set_device(0)
    precision = heom.FP64 if args.precision == "fp64" else heom.FP32_MIXED
    base = hi.fmo_like()
    dip = hi.unit_vectors(np.random.default_rng(70), 7)
    relax, emis = hi.fluorescence_runs(base["H"], dip, base["baths"], 300.0, base["depth"], 1.0,
                                       2000, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    he = heom.Hierarchy(relax, precision)
    st = he.new_state(relax["rho0"])
    he.propagate(st, 1.0, relax["n_steps"], relax["record_every"], hermitian=True)
    P = []
    for r in emis:
        hf = heom.Hierarchy(r, precision)
        y = hf.new_state()
        heom.emission_start(he, st, hf, y, r["observable"]["mu"][1:])
        rec = hf.propagate(y, 1.0, r["n_steps"], 1, r["observable"], hermitian=False)
        P.append(rec[:, 0] + 1j * rec[:, 1])
        print("fluorescence: direction %d done, %.2f s" % (len(P), time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    S = heom.spectrum(np.stack(P), 1.0, np.arange(-1000.0, 1001.0, 1.0))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = he.n_ado
    updates = n * (relax["n_steps"] + 3 * emis[0]["n_steps"])
    print(json.dumps({"workload": "fluorescence: fmo_like thermal state (2000 steps) + 3 x 1000 "
                                  "emission steps, 3060 ADOs, spectrum on 2001 points",
                      "precision": args.precision, "seconds": el,
                      "ado_updates_per_s": updates / el,
                      "peak_cm_rel": float(np.arange(-1000.0, 1001.0, 1.0)[np.argmax(S)])}),
          flush=True)


def run_absorption(args):
    """Linear absorption of the FMO-like system (3 directions, 1000 steps,
    FP64): three full (N+1)-state dipole-correlation runs against one
    coherence-block run of the three directions.  Times both."""
    import torch
    import paper_1803_03498_amd as heom
    torch.cuda.set_device(0)
    runs = hi.fmo_like_absorption()
    out = {"workload": "absorption: fmo_like, 3 directions x 1000 RK4 steps, 3060 ADOs, FP64"}
    for form in ("full", "block"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if form == "full":
            for r in runs:
                h = heom.Hierarchy(r, heom.FP64)
                st = h.new_state(r["rho0"])
                h.propagate(st, r["dt_fs"], r["n_steps"], 1, r["observable"], hermitian=False)
        else:
            r = runs[0]
            prob = {"H": r["H"][1:, 1:], "temperature_K": r["temperature_K"], "depth": r["depth"],
                    "flags": 0, "baths": [dict(b, state=b["state"] - 1) for b in r["baths"]]}
            mu3 = np.stack([q["observable"]["mu"][1:] for q in runs])
            h = heom.Hierarchy(prob, heom.FP64)
            h.propagate_block(h.block_state(mu3), r["dt_fs"], r["n_steps"], 1, mu3)
        torch.cuda.synchronize()
        out[form + "_seconds"] = time.perf_counter() - t0
        print("absorption: %s form %.3f s" % (form, out[form + "_seconds"]), file=sys.stderr,
              flush=True)
    out["bytes_per_ado_full"] = 3 * 8 * 8 * 16
    out["bytes_per_ado_block"] = 7 * 3 * 16
    print(json.dumps(out), flush=True)


def _device_copy(torch, gib, steps, warmup):
    """A plain device-to-device copy of `gib` GiB, `steps` times: (elements,
    seconds).  Bytes moved per copy: 8 per element (read + write)."""
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del src, dst
    torch.cuda.empty_cache()
    return n, el


def run_copy(args):
    """A plain device-to-device copy of known size: the reference against
    which the HBM byte counters of a profiler run are scaled."""
    import torch
    torch.cuda.set_device(0)
    steps = args.steps if args.steps is not None else 20
    warmup = args.warmup if args.warmup is not None else 3
    n, el = _device_copy(torch, args.copy_gib, steps, warmup)
    print(json.dumps({"workload": "copy", "bytes_read_per_copy": 4 * n,
                      "bytes_written_per_copy": 4 * n, "steps": steps,
                      "ms_per_copy": 1e3 * el / steps,
                      "GBps_read_plus_write": 8 * n * steps / el / 1e9}), flush=True)


def main():
    args = parse()
    if args.workload == "copy":
        run_copy(args)
        return
    if args.workload == "fluorescence":
        run_fluorescence(args)
        return
    if args.workload == "absorption":
        run_absorption(args)
        return
    if args.workload == "serve":
        if args.gpus != 1:
            print("bench.py runs on one GPU only (--gpus %d requested)" % args.gpus,
                  file=sys.stderr)
            sys.exit(2)
        run_serve(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    # the serving mix's oracle leg spawns its host processes before any GPU work
    mix_cpu = _mix_cpu_oracle(args)
    import torch

    import paper_1803_03498_amd as heom
    from paper_1803_03498_amd import _abi

    prob = WORKLOADS[args.workload]()
    precision = {"fp32_mixed": heom.FP32_MIXED, "fp32_herm": heom.FP32_HERM,
                 "fp64": heom.FP64}[args.precision]
    steps = args.steps if args.steps is not None else {"aggregate48": 50, "fmo66_pade": 20}.get(
        args.workload, 200)
    warmup = args.warmup if args.warmup is not None else 5
    torch.cuda.set_device(0)
    h = heom.Hierarchy(prob, precision)
    N, n, W_modes = h.N, h.n_ado, h.W
    info = h.info
    rec_every = prob["record_every"]
    st = h.new_state(prob["rho0"])
    work = h.workspace(max(steps, warmup), rec_every, heom.OBS_POPULATION)
    print("workload %s: N=%d W=%d D=%d n_ado=%d precision=%s state=%.2f GB" % (
        args.workload, N, h.W, prob["depth"], n, args.precision,
        (info["rest_bytes"] + info["sigma0_bytes"]) / 1e9), file=sys.stderr, flush=True)

    lib = heom.load()
    h.propagate(st, prob["dt_fs"], warmup, rec_every, hermitian=True, work=work)
    torch.cuda.synchronize()
    # the timed steps as a caller runs them (step graph replays for runs of
    # 8 steps or more): the line's value
    t0 = time.perf_counter()
    rec = h.propagate(st, prob["dt_fs"], steps, rec_every, hermitian=True, work=work)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same number of steps again with HIP events around every bulk
    # launch (direct launches): the roofline's per-launch time
    lib.heom_timing_enable(1)
    lib.heom_timing_read(None, None, None, 1)
    torch.cuda.synchronize()
    h.propagate(st, prob["dt_fs"], steps, rec_every, hermitian=True, work=work)
    torch.cuda.synchronize()
    lib.heom_timing_enable(0)
    ms = ctypes.c_double()
    launches = ctypes.c_int64()
    kbytes = ctypes.c_double()
    lib.heom_timing_read(ctypes.byref(ms), ctypes.byref(launches), ctypes.byref(kbytes), 1)

    kernel_short = _bulk_kernel_name(info, precision, N, heom)
    kernel_name = kernel_short + " (RK4 stage, ADOs u>=1)"
    traffic = measured_traffic(kernel_short, args.workload, args.precision)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / steps
    ado_updates = n * steps / elapsed
    e = info["elem_bytes"]
    step_bytes = 13.0 * ((n - 1) * N * N * e + N * N * 16)
    hbm_gbs = step_bytes * steps / elapsed / 1e9
    avg_launch_s = ms.value / 1e3 / max(launches.value, 1)
    bytes_per_launch = kbytes.value / max(launches.value, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # what a plain 4 GiB device copy (read + write) sustains on this GPU, the
    # practical ceiling of a read/write stream next to the datasheet peak
    n_copy, t_copy = _device_copy(torch, 4.0, 20, 3)
    copy_gbs = 8.0 * n_copy * 20 / t_copy / 1e9
    pops = rec[-1, :N]
    print("ms/step %.3f  ADO-updates/s %.3e  alg HBM %.0f GB/s  bulk kernel avg %.3f ms "
          "(%.0f GB/s)  trace %.15f" % (ms_per_step, ado_updates, hbm_gbs, avg_launch_s * 1e3,
                                        achieved, rec[-1, N]), file=sys.stderr, flush=True)
    if not np.all(np.isfinite(pops)):
        raise RuntimeError("non-finite populations")

    # untimed: the same steps from the initial state in FP64 (timed on its
    # own) and again in the benchmarked precision, for the error of the
    # reduced-precision result against FP64
    fp64 = None
    if precision != heom.FP64 and not args.no_fp64_check:
        del work
        fp64 = _fp64_reference(heom, torch, lib, prob, precision, steps, rec_every, N, n)
        print("FP64 %.3f ms/step; FP32 vs FP64 max population error %.3e" % (
            fp64["ms_per_step"], fp64["fp32_vs_fp64_max_population_error"]), file=sys.stderr,
            flush=True)

    cpu = None
    if args.cpu_baseline_seconds > 0:
        cpu = cpu_baseline(prob, args.cpu_baseline_seconds)

    serve = None
    if args.serve_seconds > 0:
        work = st = h = None  # the 48-site state and stage copies leave the device
        torch.cuda.empty_cache()
        serve = serve_leg(args, mix_cpu)

    line = {
        "metric": METRIC,
        "value": ado_updates,
        "unit": "ADO-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == heom.FP64 else "f32",
        "data": "synthetic",
        "hbm_GBps_algorithmic": hbm_gbs,
        "config": {
            "workload": "%s: %d sites, W=%d modes, depth %d, %d ADOs of %dx%d %s; RK4 dt=%g fs"
                        % (args.workload, N, W_modes, prob["depth"], n, N, N,
                           {heom.FP32_MIXED: "complex64 (sigma_0 complex128)",
                            heom.FP32_HERM: "Hermitian-packed real float32 (sigma_0 complex128)",
                            heom.FP64: "complex128"}[precision], prob["dt_fs"]),
            "n_ado": n, "n_states": N, "n_modes": W_modes, "depth": prob["depth"],
            "precision": args.precision, "record_every": rec_every,
            "bytes_per_step_algorithmic": step_bytes,
        },
        "roofline": {
            "kernel": kernel_name,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": avg_launch_s * 1e3,
            "bytes_per_launch_algorithmic": bytes_per_launch,
            "table_bytes_per_launch": _table_bytes_per_launch(
                kernel_short, n, W_modes, prob["depth"], precision == heom.FP64),
            "device_copy_GBps": copy_gbs,
            "frac_of_device_copy": achieved / copy_gbs,
        },
        "cpu_baseline": cpu,
        "fp64": fp64,
        "serve": serve,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
