#!/usr/bin/env python3
"""Benchmark of librr on one MI355X.

One step = every dense N-D permute of the benchmark workload, once:
  3-D 512x512x256 under all six axis orders, 4-D 64x128x128x64 under (0,3,1,2)
  and (0,2,3,1), 5-D 32^5 under (4,2,0,3,1) and the 16384x16384 transpose,
  each at element sizes 16, 8, 4, 2 and 1 bytes (50 launches, 24.25 GiB per side).
Inputs are seeded random bits already resident in HBM.  Throughput is effective
bandwidth: 2 * bytes-per-side / time (read + write, decimal GB/s).

Printed: one JSON line with the step throughput, ceilings (hipMemcpyAsync D2D
and the library's own copy kernel), the roofline of the dominant kernel from
per-launch HIP events, the oracle's CPU throughput on a bounded sample, and
side measurements of the interlace workloads, the batched launch and the
serving loop.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "permute eff. GB/s (% of D2D memcpy, % of 8 TB/s); served p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-tune", action="store_true", help="time the built-in tile shapes only")
    ap.add_argument("--tune-cache", default=None,
                    help="load tuned tile shapes from this file if it exists (no tuning launches), "
                         "else tune and save them there")
    ap.add_argument("--no-side", action="store_true", help="skip interlace/batched/serve side runs")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop side run")
    ap.add_argument("--serve-requests", type=int, default=100_000, help="most requests per arrival rate")
    ap.add_argument("--side-only", choices=("serve", "batched"), default=None,
                    help="run only this side measurement and print its JSON (no dense step)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup+steps and exit (for rocprofv3 runs)")
    ap.add_argument("--profile-odd", action="store_true",
                    help="launch each odd-shaped permute of ODD_CASES once with both sides "
                         "non-temporal, then once with the planner's cache policy, and exit "
                         "(for rocprofv3 counter runs; prints the launch order)")
    ap.add_argument("--profile-access", action="store_true",
                    help="run each index-set and range read of the access-pattern side run once "
                         "(each after a 512 MiB cache-flush write), print one JSON line per launch "
                         "in launch order and exit (for rocprofv3 kernel traces and HBM counters)")
    ap.add_argument("--profile-stencil", action="store_true",
                    help="run each stencil of the stencil side run once (each after a 512 MiB "
                         "cache-flush write), print one JSON line per launch in launch order and "
                         "exit (for rocprofv3 kernel traces and HBM counters)")
    ap.add_argument("--profile-interlace", action="store_true",
                    help="run each interlace and de-interlace workload once (each after a 512 MiB "
                         "cache-flush write), print one JSON line per launch in launch order and "
                         "exit (for rocprofv3 kernel traces and HBM counters)")
    ap.add_argument("--profile-batch", nargs="?", const="graph", default=None, choices=("graph", "serial"),
                    help="build the 4096-job batch as a tuned handle -- graph: graph-replayed with its "
                         "groups side by side (what the batch bench times); serial: its groups one after "
                         "another on one stream -- replay it three times (each after a 512 MiB "
                         "cache-flush write), print the handle's groups (bytes per side each) and the "
                         "replay times, and exit (for rocprofv3 kernel traces and HBM counters of the "
                         "kernel groups: the replays are the last 3 x groups dispatches)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="turn the counter_collection.csv files of two rocprofv3 --pmc runs of "
                         "'--profile-only --steps 1 --warmup 0' (FETCH_SIZE, then WRITE_SIZE) into "
                         "profiles/counters.json, calibrated on the step's plain copies; no GPU needed")
    return ap.parse_args()


# The counter runs that --ingest-counters expects (one dispatch per case, tuned
# shapes loaded from the cache the timed run wrote).
PMC_COMMANDS = [
    "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- "
    "python3 bench.py --profile-only --steps 1 --warmup 0 --tune-cache <cache>",
    "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- "
    "python3 bench.py --profile-only --steps 1 --warmup 0 --tune-cache <cache>",
]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("rr_device.hpp", "rr_kernels.hip", "rr_plan.cpp", "rr_plan.hpp"):
        with open(os.path.join(ROOT, "paper_1011_3583_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def dense_cases():
    """(name, dims, perm, elem_size, bytes per side) of every launch of one step."""
    import rr_synth
    cases = []
    for name, dims, perm in rr_synth.DENSE_CASES:
        for e in sorted(rr_synth.ESIZES, reverse=True):
            n = 1
            for d in dims:
                n *= d
            cases.append((name, dims, perm, e, n * e))
    return cases


# Consecutive launches of the step read and write places this far apart (modulo
# the buffers), so no case finds its input or output lines still in the 256 MB
# Infinity Cache from the launches just before it.
STEP_STRIDE = 768 << 20


def step_addresses(pool: int, out: int, max_nb: int, i: int, nb: int):
    """(src, dst) of case i: the input somewhere in the two-region pool (2 * max_nb
    bytes), the output somewhere in out (max_nb bytes), both 4 KiB aligned and
    STEP_STRIDE further on than case i-1's (wrapping)."""
    def at(base, size, k):
        room = size - nb
        return base + ((k * STEP_STRIDE) % (room + 1)) // 4096 * 4096 if room > 0 else base
    return at(pool, 2 * max_nb, i), at(out, max_nb, i + 1)


def _pmc_rows(path: str, counter: str):
    """(dispatch id, kernel name as k_x<a,b>, counter KiB) of the library's kernels."""
    import csv
    out = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"]
            if r["Counter_Name"] != counter or not name.startswith("void rr::k_"):
                continue
            out.append((int(r["Dispatch_Id"]), name[len("void rr::"):].split("(")[0].replace(" ", ""),
                        float(r["Counter_Value"])))
    out.sort()
    return out


def ingest_counters(fetch_csv: str, write_csv: str, out_path: str | None = None) -> dict:
    """HBM bytes per launch of each kernel of the step, from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what it reads for the step's
    plain copies (identity permutes: k_copy, a known number of bytes each way)."""
    cases = dense_cases()
    f = _pmc_rows(fetch_csv, "FETCH_SIZE")
    w = _pmc_rows(write_csv, "WRITE_SIZE")
    n = len(cases)
    if not f or len(f) % n or len(w) != len(f):
        raise SystemExit(f"expected a multiple of {n} library dispatches in each run, got {len(f)} and {len(w)}")
    for (_, kf, _), (_, kw, _) in zip(f, w):
        if kf != kw:
            raise SystemExit(f"the two runs launched different kernels ({kf} vs {kw})")
    algo = [cases[i % n][4] for i in range(len(f))]
    copies = [i for i in range(len(f)) if f[i][1].startswith("k_copy")]
    if not copies:
        raise SystemExit("no plain copy in the step to calibrate against")
    rf = sum(algo[i] for i in copies) / sum(f[i][2] * 1024 for i in copies)
    wf = sum(algo[i] for i in copies) / sum(w[i][2] * 1024 for i in copies)
    kernels = {}
    for i, (_, k, fk) in enumerate(f):
        e = kernels.setdefault(k, {"launches": 0, "algorithmic": 0.0, "fetch": 0.0, "write": 0.0})
        e["launches"] += 1
        e["algorithmic"] += 2 * algo[i]
        e["fetch"] += fk * 1024 * rf
        e["write"] += w[i][2] * 1024 * wf
    out = {}
    for k, e in sorted(kernels.items()):
        m = e["launches"]
        hbm = (e["fetch"] + e["write"]) / m
        out[k] = {"launches": m, "algorithmic_bytes_per_launch": round(e["algorithmic"] / m),
                  "read_bytes_per_launch": round(e["fetch"] / m), "write_bytes_per_launch": round(e["write"] / m),
                  "hbm_bytes_per_launch": round(hbm), "traffic_over_algorithmic": round(hbm / (e["algorithmic"] / m), 4)}
    prof = {"source_hash": kernel_source_hash(), "commands": PMC_COMMANDS,
            "calibration": {"kernel": "k_copy (identity permutes of the step)", "launches": len(copies),
                            "fetch_scale": round(rf, 5), "write_scale": round(wf, 5)},
            "kernels": out}
    if out_path is None:
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        out_path = os.path.join(ROOT, "profiles", "counters.json")
    with open(out_path, "w") as fh:
        json.dump(prof, fh, indent=1)
    return prof


def kernel_name(d: dict) -> str:
    if d["class"] == "tile":
        return f"k_tile<{d['unit']},{d['g']}>"
    if d["class"] == "run":
        return f"k_run<{d['vec']}>"
    if d["class"] == "copy":
        return f"k_copy<{d['vec']}>"
    if d["class"] == "weave":
        return f"k_weave<{d['unit']},{d['n']},{d['de']},{d['chunks']}>"
    return d["class"]


# Permutes whose tile rows start inside 128-byte lines (odd extents), 2^28 bytes
# per side or so: (dims, perm, element bytes).
ODD_CASES = [((8191, 4097), (1, 0), 8), ((999, 1001, 61), (2, 1, 0), 4), ((32761, 4097), (1, 0), 2),
             ((4095, 4097), (1, 0), 16), ((4325, 1001, 31), (2, 0, 1), 2)]


def profile_odd():
    """One launch per (case, policy): both sides non-temporal, then the planner's
    own choice (cached stores and XCD tile ranges where rows share lines)."""
    import torch
    import paper_1011_3583_amd as rr
    rr.lib()
    sh = torch.cuda.current_stream().cuda_stream
    nmax = max(int(__import__("numpy").prod(d)) * e for d, _, e in ODD_CASES)
    src = torch.empty(nmax, dtype=torch.uint8, device="cuda")
    src.random_(0, 256)
    dst = torch.empty(nmax, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for dims, perm, e in ODD_CASES:
        for name, kw in (("streamed", dict(cache=0, xcd=False)), ("planner", {})):
            rr.set_tile_override(**kw)
            d = rr.plan_describe(dims, perm, e, dst.data_ptr(), src.data_ptr())
            rr.check(rr.permute_raw(dst.data_ptr(), src.data_ptr(), dims, perm, e, sh))
            torch.cuda.synchronize()
            print(json.dumps({"dims": dims, "perm": perm, "esize": e, "policy": name, "flags": int(d["flags"]),
                              "kernel": kernel_name(d)}), flush=True)
    rr.set_tile_override()


def main():
    args = parse()
    if args.ingest_counters:
        print(json.dumps(ingest_counters(*args.ingest_counters), indent=1))
        return
    if args.profile_odd:
        profile_odd()
        return
    if args.profile_batch:
        profile_batch(args.profile_batch)
        return
    if args.profile_access:
        profile_access()
        return
    if args.profile_stencil:
        profile_stencil()
        return
    if args.profile_interlace:
        profile_interlace()
        return
    if args.side_only:
        import torch
        import paper_1011_3583_amd as rr
        import rr_synth
        rr.lib()
        torch.cuda.set_device(0)
        if args.side_only == "serve":
            out = bench_serve(rr, rr_synth, torch, args.serve_requests)
        else:
            out = bench_batched(rr, rr_synth, torch, torch.cuda.current_stream())
        print(json.dumps({args.side_only: out}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library "
              f"has no multi-GPU path (each GPU would run its own share of the jobs).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1011_3583_amd as rr
    import rr_synth

    # the CPU baseline forks its worker processes, so it runs before anything
    # touches the GPU
    cpu = None if (args.no_cpu or args.profile_only) else cpu_baseline()
    rr.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    cases = dense_cases()
    max_nb = max(c[4] for c in cases)
    pool = torch.empty(2 * max_nb, dtype=torch.uint8, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(1011_3583)
    for i in range(0, pool.numel(), 1 << 30):
        pool[i:i + (1 << 30)].random_(0, 256, generator=g)
    out = torch.empty(max_nb, dtype=torch.uint8, device=dev)
    plans = []
    for i, (name, dims, perm, e, nb) in enumerate(cases):
        src, dst = step_addresses(pool.data_ptr(), out.data_ptr(), max_nb, i, nb)
        d = rr.plan_describe(dims, perm, e, dst, src)
        plans.append((src, kernel_name(d), dst))

    def retag():
        plans[:] = [(p[0], kernel_name(rr.plan_describe(c[1], c[2], c[3], p[2], p[0])), p[2])
                    for p, c in zip(plans, cases)]

    def step(events=None, only=None):
        """One pass of the 50 permutes; with `events`, a pair of HIP events brackets
        each launch (of kernel `only` alone when given)."""
        for i, (name, dims, perm, e, nb) in enumerate(cases):
            src, dst = plans[i][0], plans[i][2]
            ev = events is not None and (only is None or plans[i][1] == only)
            if ev:
                events[i][0].record(stream)
            st = rr.permute_raw(dst, src, dims, perm, e, sh)
            if st != 0:
                raise rr.RRError(st, rr.last_error())
            if ev:
                events[i][1].record(stream)

    def new_events():
        return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]

    def instrumented_pass(nsteps):
        """Per-launch HIP-event times (ms) of nsteps untimed steps: [case][step]."""
        evs = [new_events() for _ in range(nsteps)]
        for k in range(nsteps):
            step(evs[k])
        torch.cuda.synchronize()
        return [[evs[k][i][0].elapsed_time(evs[k][i][1]) for k in range(nsteps)] for i in range(len(cases))]

    def kernel_of_most_time(per_case_ms):
        tot = {}
        for i, ms in enumerate(per_case_ms):
            tot[plans[i][1]] = tot.get(plans[i][1], 0.0) + sum(ms)
        return max(tot, key=tot.get)

    # untuned pass (built-in tile shapes), for reference
    untuned_ms = None
    cached = bool(args.tune_cache) and os.path.exists(args.tune_cache) and not args.no_tune
    if cached:
        rr.tune_load(args.tune_cache)
        retag()
    elif not args.no_tune:
        rr.tune_clear()
        step()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step()
        b.record(stream)
        b.synchronize()
        untuned_ms = a.elapsed_time(b)
        # autotune every case once (runs each candidate tile shape; cached for the timed steps)
        for i, (name, dims, perm, e, nb) in enumerate(cases):
            rr.tune_permute(plans[i][2], plans[i][0], dims, perm, e, sh)
        retag()
        if args.tune_cache:
            rr.tune_save(args.tune_cache)
    # Warm-up: the first step is instrumented (every launch between HIP events) to
    # find the kernel with the most time; the timed steps then bracket only that
    # kernel's launches, since 100 event records per step cost ~4 % of it.
    dom = None
    for w in range(args.warmup):
        if w == 0 and not args.profile_only:
            dom = kernel_of_most_time(instrumented_pass(1))
        else:
            step()
    torch.cuda.synchronize()
    if args.profile_only:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return

    evs = [new_events() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s], only=dom)      # dom None (no warm-up): every launch
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    bytes_per_step = sum(2 * c[4] for c in cases)
    value = bytes_per_step * args.steps / wall / 1e9

    # the dominant kernel's launches, timed live inside the timed steps
    timed_ms = [[evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(args.steps)]
                if dom is None or plans[i][1] == dom else None for i in range(len(cases))]
    if dom is None:
        dom = kernel_of_most_time(timed_ms)
    dk = {"bytes": 0, "ms": 0.0, "launches": 0}
    for i, c in enumerate(cases):
        if plans[i][1] == dom:
            dk["bytes"] += 2 * c[4] * args.steps
            dk["ms"] += sum(timed_ms[i])
            dk["launches"] += args.steps
    achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9

    # every launch's duration, from an instrumented pass after the timed steps
    per_case_ms = instrumented_pass(max(1, min(args.steps, 3)))
    nsteps_detail = len(per_case_ms[0])
    detail = {}
    by_kernel = {}
    for i, (name, dims, perm, e, nb) in enumerate(cases):
        ms = sorted(per_case_ms[i])[len(per_case_ms[i]) // 2]
        key = f"{name} {tuple(perm)} e{e}"
        detail[key] = round(2 * nb / (ms * 1e-3) / 1e9, 1)
        k = plans[i][1]
        agg = by_kernel.setdefault(k, {"bytes": 0, "ms": 0.0, "launches": 0})
        agg["bytes"] += 2 * nb * nsteps_detail
        agg["ms"] += sum(per_case_ms[i])
        agg["launches"] += nsteps_detail
    kernel_time_ms = sum(sum(v) for v in per_case_ms) / nsteps_detail
    traffic = None
    prof_path = os.path.join(ROOT, "profiles", "counters.json")
    if os.path.exists(prof_path):
        with open(prof_path) as fh:
            prof = json.load(fh)
        entry = prof.get("kernels", {}).get(dom)
        if entry and prof.get("source_hash") == kernel_source_hash():
            traffic = entry.get("hbm_bytes_per_launch")

    # ceilings: hipMemcpyAsync D2D and the library's copy kernel, 1 GiB per side
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_void_p]
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)

    def timed(fn, reps=7):
        ts = []
        for r in range(reps + 2):
            flush.fill_(r & 0xff)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        ts = sorted(ts[2:])
        return ts[len(ts) // 2]

    # Ceilings at every per-side size of the step, same protocol (cache flush, HIP
    # events around one launch, median): hipMemcpyAsync D2D (the runtime's blit
    # kernel) and the library's own copy kernel.  Each case is compared with the
    # better of the two at its own size; the step with the time it would take if
    # every case ran at that ceiling.
    ceilings = {}
    for nb in sorted({c[4] for c in cases}):
        t_d2d = timed(lambda: hip.hipMemcpyAsync(out.data_ptr(), pool.data_ptr(), nb, 3, sh), 5)
        t_cpy = timed(lambda: rr.check(rr.permute_raw(out.data_ptr(), pool.data_ptr(), (nb,), (0,), 1, sh)), 5)
        ceilings[nb] = {"d2d": 2 * nb / t_d2d / 1e9, "rr_copy": 2 * nb / t_cpy / 1e9}
    best_copy = {nb: max(v.values()) for nb, v in ceilings.items()}
    step_time_at = lambda key: sum(2 * c[4] / ((ceilings[c[4]][key] if key else best_copy[c[4]]) * 1e9)
                                   for c in cases)   # seconds
    d2d = bytes_per_step / step_time_at("d2d") / 1e9           # the step at D2D speed, size by size
    rrcopy = bytes_per_step / step_time_at("rr_copy") / 1e9
    bestc = bytes_per_step / step_time_at(None) / 1e9
    pct_case = {f"{n} {tuple(p)} e{e}": round(100 * detail[f"{n} {tuple(p)} e{e}"] / best_copy[nb], 1)
                for n, d, p, e, nb in cases}
    # the small case: 1024 x 1024 4-byte transpose, 4 MiB per side -- resident in
    # the caches when repeated back to back (warm), and from a flushed cache (cold)
    sd, sp, se = rr_synth.SMALL_CASE[1], rr_synth.SMALL_CASE[2], rr_synth.SMALL_CASE[3]
    snb = 1024 * 1024 * se
    run_small = lambda: rr.check(rr.permute_raw(out.data_ptr(), pool.data_ptr(), sd, sp, se, sh))
    for _ in range(5):
        run_small()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(50):
        run_small()
    b.record(stream)
    b.synchronize()
    t_warm = a.elapsed_time(b) * 1e-3 / 50
    t_cold = timed(run_small, 7)
    small_case = {"workload": "2-D 1024x1024 4-byte transpose (1,0), 4 MiB per side",
                  "warm_cache_resident_GBps": round(2 * snb / t_warm / 1e9, 1),
                  "cold_GBps": round(2 * snb / t_cold / 1e9, 1),
                  "note": "cache-resident: 4 MiB per side fits the L2 and the 256 MB Infinity Cache, so the "
                          "warm figure is not an HBM rate; cold = after a 512 MiB flush, HIP events around one "
                          "launch (launch overhead included)"}

    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic: seeded random bits, resident in HBM",
        "config": {
            "workload": "dense N-D permutes: 3-D 512x512x256 all 6 orders, 4-D 64x128x128x64 "
                        "(0,3,1,2),(0,2,3,1), 5-D 32^5 (4,2,0,3,1), 2-D 16384x16384 (1,0); "
                        "element sizes 16,8,4,2,1 bytes",
            "launches_per_step": len(cases),
            "bytes_per_side_per_step": bytes_per_step // 2,
        },
        "pct_of_d2d_memcpy": round(100 * value / d2d, 1),
        "pct_of_best_copy": round(100 * value / bestc, 1),
        "pct_of_rr_copy": round(100 * value / rrcopy, 1),
        "pct_of_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 1),
        "kernel_only_GBps": round(bytes_per_step / (kernel_time_ms * 1e-3) / 1e9, 1),
        "instrumentation": "timed steps: HIP events around the dominant kernel's launches only; "
                           "kernels / detail_GBps / kernel_only_GBps: a separate pass with every "
                           "launch between events",
        "autotuned": not args.no_tune,
        "untuned_step_GBps": round(bytes_per_step / (untuned_ms * 1e-3) / 1e9, 1) if untuned_ms else None,
        "ceilings_GBps": {"step_at_d2d_hipMemcpyAsync": round(d2d, 1), "step_at_rr_copy": round(rrcopy, 1),
                          "step_at_best_copy": round(bestc, 1), "hbm_peak": HBM_PEAK_GBPS,
                          "by_bytes_per_side": {str(nb): {k: round(v, 1) for k, v in c.items()}
                                                for nb, c in sorted(ceilings.items())},
                          "protocol": "512 MiB cache-flush write before each run, HIP events around one "
                                      "launch, median of 5; per size, hipMemcpyAsync D2D and the library's "
                                      "copy kernel; step_at_x = step bytes / (sum over cases of 2 * bytes / "
                                      "ceiling at the case's size)"},
        "pct_of_best_copy_by_case": pct_case,
        "small_case": small_case,
        "cache_state": "timed steps: each case reads and writes lines 768 MiB away from the launches just "
                       "before it (no input or output of a case is in the 256 MB Infinity Cache when it "
                       "starts); no flush inside the timed region",
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "launches": dk["launches"],
                     "avg_launch_us": round(dk["ms"] / dk["launches"] * 1e3, 2),
                     "algorithmic_bytes_per_launch": dk["bytes"] // dk["launches"]},
        "kernels": {k: {"GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1),
                        "avg_launch_us": round(v["ms"] / v["launches"] * 1e3, 2),
                        "launches": v["launches"]} for k, v in sorted(by_kernel.items())},
        "detail_GBps": detail,
        "kernel_source": kernel_source_hash(),
        "device": {"name": torch.cuda.get_device_name(0),
                   "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", None),
                   "hip": torch.version.hip, "library": rr.lib().rr_version().decode()},
    }
    if not args.no_side:
        side = {}
        try:
            side["interlace"] = bench_interlace(rr, rr_synth, pool, out, stream, timed)
        except Exception as ex:  # side measurements never hide the main line
            side["interlace"] = {"error": str(ex)}
        try:
            side["reorder"] = bench_reorder(rr, pool, out, stream, timed)
        except Exception as ex:
            side["reorder"] = {"error": str(ex)}
        try:
            side["access_patterns"] = bench_access_patterns(rr, torch, pool, out, stream, timed)
        except Exception as ex:
            side["access_patterns"] = {"error": str(ex)}
        try:
            side["stencil"] = bench_stencil(rr, rr_synth, pool, out, stream, timed)
        except Exception as ex:
            side["stencil"] = {"error": str(ex)}
        try:
            side["paper_tables"] = bench_paper_tables(rr, rr_synth, pool, out, stream, timed)
        except Exception as ex:
            side["paper_tables"] = {"error": str(ex)}
        del pool, out, flush
        torch.cuda.empty_cache()
        try:
            side["batched"] = bench_batched(rr, rr_synth, torch, stream)
        except Exception as ex:
            side["batched"] = {"error": repr(ex)}
        torch.cuda.empty_cache()
        if not args.no_serve:
            try:
                side["serve"] = bench_serve(rr, rr_synth, torch, args.serve_requests)
            except Exception as ex:
                side["serve"] = {"error": repr(ex)}
        result["side"] = side

    if cpu is not None:
        result["cpu_baseline"] = cpu

    print(json.dumps(result), flush=True)


# N-to-M reorders (base and range): name, input dims, base, range, order, element bytes
REORDER_CASES = [
    ("crop_transpose_3d", (512, 512, 256), (16, 16, 0), (480, 480, 256), (2, 0, 1), 4),
    ("nhwc_to_nchw_batch_slice", (64, 128, 128, 64), (8, 0, 0, 0), (48, 128, 128, 64), (0, 3, 1, 2), 2),
    ("fixed_axis_4d", (4, 16, 2048, 2048), (0, 5, 0, 0), (4, 1, 2048, 2048), (2, 0, 3), 4),
    ("row_slab", (16384, 16384), (4096, 0), (8192, 16384), (0, 1), 4),
    ("hwc_channel_2", (16384, 16384, 4), (0, 0, 2), (16384, 16384, 1), (0, 1), 1),
]


def bench_reorder(rr, pool, out, stream, timed):
    """Effective GB/s (2 x output bytes / time) of N-to-M reorders of pool data; the
    plan class says whether the box tiled, copied or had to gather."""
    res = {}
    for name, dims, base, rng, order, e in REORDER_CASES:
        nout = 1
        for o in order:
            nout *= rng[o]
        nin = e
        for d in dims:
            nin *= d
        assert nin <= pool.numel() and nout * e <= out.numel()
        src = pool.data_ptr()
        d = rr.reorder_describe(dims, base, rng, order, e, out.data_ptr(), src)
        t = timed(lambda: rr.check(rr.reorder_raw(out.data_ptr(), src, dims, base, rng, order, e, stream.cuda_stream)), 5)
        res[name] = {"GBps": round(2 * nout * e / t / 1e9, 1), "class": d["class"],
                     "out_bytes": nout * e, "kernel": kernel_name(d)}
    return res


def bench_access_patterns(rr, torch, pool, out, stream, timed):
    """Index-set and range reads of pool data (a 1 GiB table): GB/s counts the
    algorithmic bytes (indices read + elements read + elements written)."""
    res = {}
    sh = stream.cuda_stream
    table = 1 << 30
    g = torch.Generator(device=pool.device)
    g.manual_seed(3583)
    count = 1 << 26
    for e in (4, 16):
        n = table // e
        idx = torch.randint(0, n, (count,), generator=g, device=pool.device, dtype=torch.int64)
        for name, ix in (("random", idx), ("sorted", torch.sort(idx).values)):
            t = timed(lambda: rr.check(rr.gather_raw(out.data_ptr(), pool.data_ptr(), n, ix.data_ptr(), count, e, 0,
                                                     sh)), 5)
            res[f"gather_{name}_e{e}"] = {"GBps": round(count * (8 + 2 * e) / t / 1e9, 1), "elements": count}
        del idx
        for stride in (2, -1, 7):
            start = 0 if stride > 0 else n - 1
            cnt = min(count, (n - 1) // abs(stride) + 1)
            t = timed(lambda: rr.check(rr.copy_range_raw(out.data_ptr(), pool.data_ptr(), n, start, stride, cnt, e,
                                                         sh)), 5)
            res[f"range_stride{stride}_e{e}"] = {"GBps": round(2 * cnt * e / t / 1e9, 1), "elements": cnt}
    return res


# The paper's own results on a Tesla C1060 (GB/s, read + write): Table 1
# (3D permute of 128x256x512 floats; its memcpy row is 77.82), Table 2 (reorder)
# and Table 3 (interlace / de-interlace of n arrays).  Context only.
PAPER_MEMCPY_GBPS = 77.82
PAPER_TABLE1 = {(0, 2, 1): 62.55, (1, 0, 2): 63.17, (1, 2, 0): 57.38, (2, 0, 1): 59.63, (2, 1, 0): 58.42}
PAPER_TABLE2 = {(1, 0, 2): 76.00, (1, 0, 2, 3): 75.41, (3, 2, 0, 1): 56.24, (3, 0, 2, 1, 4): 43.40}
PAPER_TABLE3 = {4: (70.93, 68.87), 5: (73.95, 68.50), 6: (71.51, 67.61), 7: (72.14, 60.21), 8: (58.58, 60.55),
                9: (70.60, 58.25)}


def bench_paper_tables(rr, rr_synth, pool, out, stream, timed):
    """The paper's Table 1-3 workloads (4-byte elements, its fastest-first order
    notation), as % of this box's hipMemcpyAsync D2D copy of the same bytes (same
    protocol) next to the paper's % of its memcpy."""
    import ctypes
    sh = stream.cuda_stream
    res = {}
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    d2d_at = {}

    def row(gbps, paper, nb):
        if nb not in d2d_at:
            d2d_at[nb] = 2 * nb / timed(lambda: hip.hipMemcpyAsync(out.data_ptr(), pool.data_ptr(), nb, 3, sh), 5) / 1e9
        return {"GBps": round(gbps, 1), "pct_of_d2d": round(100 * gbps / d2d_at[nb], 1),
                "d2d_GBps_same_bytes": round(d2d_at[nb], 1),
                "paper_GBps_C1060": paper, "paper_pct_of_memcpy": round(100 * paper / PAPER_MEMCPY_GBPS, 1)}

    sizes = rr_synth.PAPER_TABLE1_SIZES
    dims = tuple(reversed(sizes))
    for order, paper in PAPER_TABLE1.items():
        perm = rr.order_to_perm(order)
        nb = 4 * sizes[0] * sizes[1] * sizes[2]
        t = timed(lambda: rr.check(rr.permute_raw(out.data_ptr(), pool.data_ptr(), dims, perm, 4, sh)), 5)
        res[f"table1_{''.join(map(str, order))}"] = row(2 * nb / t / 1e9, paper, nb)
    for sz, order in rr_synth.PAPER_TABLE2:
        dims = tuple(reversed(sz))
        perm = rr.order_to_perm(order)
        nb = 4
        for d in sz:
            nb *= d
        t = timed(lambda: rr.check(rr.permute_raw(out.data_ptr(), pool.data_ptr(), dims, perm, 4, sh)), 5)
        res[f"table2_{''.join(map(str, order))}"] = row(2 * nb / t / 1e9, PAPER_TABLE2[tuple(order)], nb)
    count = 1 << 24
    for n, (pi, pd) in PAPER_TABLE3.items():
        planes = [pool.data_ptr() + c * count * 4 for c in range(n)]
        ti = timed(lambda: rr.check(rr.interlace_raw(out.data_ptr(), planes, count, 4, sh)), 5)
        td = timed(lambda: rr.check(rr.deinterlace_raw(planes, out.data_ptr(), count, 4, sh)), 5)
        res[f"table3_interlace_{n}"] = row(2 * n * count * 4 / ti / 1e9, pi, n * count * 4)
        res[f"table3_deinterlace_{n}"] = row(2 * n * count * 4 / td / 1e9, pd, n * count * 4)
    return res


def bench_stencil(rr, rr_synth, pool, out, stream, timed):
    """2-D stencils on float grids of pool data: FD orders I-IV (star) and 3x3 /
    5x5 boxes on Table 4's 4096 x 4096 grid and on 16384 x 16384; GB/s counts one
    read and one write of the grid (the paper's accounting)."""
    res = {}
    g = rr_synth.rng(4)
    for rows, cols in rr_synth.STENCIL_GRIDS:
        nb = rows * cols * 4
        assert nb <= pool.numel() and nb <= out.numel()
        cases = [(f"fd_order{r}", r, c, 0) for r, c in rr_synth.FD_LAPLACIAN.items()]
        cases += [(f"box{2 * r + 1}x{2 * r + 1}", r, g.uniform(-1, 1, (2 * r + 1) ** 2).astype("float32"), 1)
                  for r in (1, 2)]
        for name, r, w, shape in cases:
            t = timed(lambda: rr.check(rr.stencil2d_raw(out.data_ptr(), pool.data_ptr(), rows, cols, r, w, shape,
                                                        stream.cuda_stream)), 5)
            res[f"{rows}x{cols}_{name}"] = round(2 * nb / t / 1e9, 1)
    return res


def bench_interlace(rr, rr_synth, pool, out, stream, timed):
    res = {}
    for name, n, count, e in rr_synth.INTERLACE_CASES:
        pb = count * e
        planes = [pool.data_ptr() + c * pb for c in range(n)]
        t1 = timed(lambda: rr.check(rr.interlace_raw(out.data_ptr(), planes, count, e, stream.cuda_stream)), 5)
        t2 = timed(lambda: rr.check(rr.deinterlace_raw(planes, out.data_ptr(), count, e, stream.cuda_stream)), 5)
        res[name] = {"interlace_GBps": round(2 * n * pb / t1 / 1e9, 1),
                     "deinterlace_GBps": round(2 * n * pb / t2 / 1e9, 1)}
    return res


def _job_buffers(torch, specs, dev="cuda"):
    """One source and one destination allocation holding every job at 256-byte offsets."""
    sizes = [int(__import__("numpy").prod(s["dims"])) * s["esize"] for s in specs]
    offs, acc = [], 0
    for n in sizes:
        offs.append(acc)
        acc += (n + 255) // 256 * 256
    src = torch.empty(acc + 256, dtype=torch.uint8, device=dev)
    dst = torch.empty(acc + 256, dtype=torch.uint8, device=dev)
    for i in range(0, src.numel(), 1 << 30):
        src[i:i + (1 << 30)].random_(0, 256)
    return src, dst, offs, sizes


def profile_access():
    """The access-pattern side run's index-set and range reads of a 1 GiB table, one
    launch each from cold caches; one JSON line per launch (name, element size,
    elements, algorithmic bytes = indices read + elements read + elements written)."""
    import torch
    import paper_1011_3583_amd as rr
    rr.lib()
    sh = torch.cuda.current_stream().cuda_stream
    table, count = 1 << 30, 1 << 26
    pool = torch.empty(table, dtype=torch.uint8, device="cuda")
    pool.random_(0, 256)
    out = torch.empty(count * 16, dtype=torch.uint8, device="cuda")
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(3583)

    def launch(name, e, n_el, alg, fn):
        flush.fill_(1)
        torch.cuda.synchronize()
        fn()
        torch.cuda.synchronize()
        print(json.dumps({"case": name, "esize": e, "elements": n_el, "algorithmic_bytes": alg}), flush=True)

    for e in (4, 16):
        n = table // e
        idx = torch.randint(0, n, (count,), generator=g, device="cuda", dtype=torch.int64)
        for name, ix in (("random", idx), ("sorted", torch.sort(idx).values)):
            launch(f"gather_{name}_e{e}", e, count, count * (8 + 2 * e),
                   lambda: rr.check(rr.gather_raw(out.data_ptr(), pool.data_ptr(), n, ix.data_ptr(), count, e, 0,
                                                  sh)))
        del idx
        for stride in (2, -1, 7):
            start = 0 if stride > 0 else n - 1
            cnt = min(count, (n - 1) // abs(stride) + 1)
            launch(f"range_stride{stride}_e{e}", e, cnt, 2 * cnt * e,
                   lambda: rr.check(rr.copy_range_raw(out.data_ptr(), pool.data_ptr(), n, start, stride, cnt, e,
                                                      sh)))


def profile_stencil():
    """The stencil side run's cases (FD orders I-IV, 3x3 and 5x5 boxes on 4096^2 and
    16384^2 float grids), one launch each from cold caches; one JSON line per launch
    (algorithmic bytes = one read and one write of the grid)."""
    import torch
    import rr_synth
    import paper_1011_3583_amd as rr
    rr.lib()
    sh = torch.cuda.current_stream().cuda_stream
    nmax = max(r * c for r, c in rr_synth.STENCIL_GRIDS)
    src = torch.randn(nmax, dtype=torch.float32, device="cuda")
    dst = torch.empty(nmax, dtype=torch.float32, device="cuda")
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    g = rr_synth.rng(4)
    for rows, cols in rr_synth.STENCIL_GRIDS:
        cases = [(f"fd_order{r}", r, c, 0) for r, c in rr_synth.FD_LAPLACIAN.items()]
        cases += [(f"box{2 * r + 1}x{2 * r + 1}", r, g.uniform(-1, 1, (2 * r + 1) ** 2).astype("float32"), 1)
                  for r in (1, 2)]
        for name, r, w, shape in cases:
            flush.fill_(1)
            torch.cuda.synchronize()
            rr.check(rr.stencil2d_raw(dst.data_ptr(), src.data_ptr(), rows, cols, r, w, shape, sh))
            torch.cuda.synchronize()
            print(json.dumps({"case": f"{rows}x{cols}_{name}", "radius": r, "shape": shape,
                              "algorithmic_bytes": 2 * rows * cols * 4}), flush=True)


def profile_interlace():
    """The interlace workloads (n planes of count elements joined set index fastest,
    and split back), one launch each from cold caches; one JSON line per launch
    (algorithmic bytes = every plane read and written once)."""
    import torch
    import rr_synth
    import paper_1011_3583_amd as rr
    rr.lib()
    sh = torch.cuda.current_stream().cuda_stream
    nmax = max(n * count * e for _, n, count, e in rr_synth.INTERLACE_CASES)
    pool = torch.empty(nmax, dtype=torch.uint8, device="cuda")
    pool.random_(0, 256)
    out = torch.empty(nmax, dtype=torch.uint8, device="cuda")
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    for name, n, count, e in rr_synth.INTERLACE_CASES:
        pb = count * e
        planes = [pool.data_ptr() + c * pb for c in range(n)]
        for op, fn in (("interlace", lambda: rr.interlace_raw(out.data_ptr(), planes, count, e, sh)),
                       ("deinterlace", lambda: rr.deinterlace_raw(planes, out.data_ptr(), count, e, sh))):
            flush.fill_(1)
            torch.cuda.synchronize()
            rr.check(fn())
            torch.cuda.synchronize()
            d = rr.interlace_describe(out.data_ptr(), planes, count, e, op == "deinterlace")
            print(json.dumps({"case": f"{name}_{op}", "n": n, "esize": e, "algorithmic_bytes": 2 * n * pb,
                              "class": d["class"], "flags": int(d.get("flags", 0))}), flush=True)


def profile_batch(mode: str = "graph"):
    """The batch bench's tuned handle (graph-replayed, groups side by side; or with
    its groups one after another on one stream), replayed three times from cold
    caches; one JSON line with the handle's choices and groups (in storage order,
    which is the launch order of a serial handle), one per replay (wall time)."""
    import torch
    import rr_synth
    import paper_1011_3583_amd as rr
    rr.lib()
    specs = rr_synth.sample_jobs(4096_0001, njobs=4096)
    src, dst, offs, sizes = _job_buffers(torch, specs)
    stream = torch.cuda.Stream()
    jobs = rr.make_jobs([(dst.data_ptr() + o, src.data_ptr() + o, s["dims"], s["perm"], s["esize"])
                         for o, s in zip(offs, specs)])
    flags = rr.RR_BATCH_TUNE | (rr.RR_BATCH_GRAPH if mode == "graph" else rr.RR_BATCH_SERIAL)
    b = rr.Batch(jobs, flags)
    print(json.dumps({"mode": mode, "batch": b.info(), "groups": b.groups()}), flush=True)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    for i in range(3):
        flush.fill_(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.launch(stream)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        print(json.dumps({"replay": i, "ms": round(t * 1e3, 3), "GBps": round(2 * sum(sizes) / t / 1e9, 1)}),
              flush=True)
    b.close()


def bench_batched(rr, rr_synth, torch, stream):
    """4096 uneven permutes: one rr_permute per job vs one batched call vs a reusable,
    autotuned handle replayed through a hipGraph (wall clock, median of runs)."""
    specs = rr_synth.sample_jobs(4096_0001, njobs=4096)
    src, dst, offs, sizes = _job_buffers(torch, specs)
    sh = stream.cuda_stream
    jobs = rr.make_jobs([(dst.data_ptr() + o, src.data_ptr() + o, s["dims"], s["perm"], s["esize"])
                         for o, s in zip(offs, specs)])
    total = sum(sizes)

    def wall(fn, reps=5):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts = sorted(ts[1:])
        return ts[len(ts) // 2]

    def per_job():
        for i, s in enumerate(specs):
            rr.check(rr.permute_raw(jobs[i].dst, jobs[i].src, s["dims"], s["perm"], s["esize"], sh))

    t_per = wall(per_job, 3)
    t_oneshot = wall(lambda: rr.check(rr.permute_batched_raw(jobs, len(specs), sh)))
    plain = rr.Batch(jobs, 0)
    t_plain = wall(lambda: plain.launch(stream))
    tuned = rr.Batch(jobs, rr.RR_BATCH_TUNE | rr.RR_BATCH_GRAPH)
    t_tuned = wall(lambda: tuned.launch(stream))
    info = tuned.info()
    plain.close()
    tuned.close()
    gbps = lambda t: round(2 * total / t / 1e9, 1)
    return {
        "jobs": len(specs), "bytes_per_side": total, "groups": info["ngroups"],
        "per_job_rr_permute_GBps": gbps(t_per), "per_job_ms": round(t_per * 1e3, 2),
        "batched_call_GBps": gbps(t_oneshot), "batched_call_ms": round(t_oneshot * 1e3, 2),
        "batch_handle_GBps": gbps(t_plain),
        "batch_handle_tuned_graph_GBps": gbps(t_tuned), "batch_handle_tuned_graph_ms": round(t_tuned * 1e3, 2),
        "tuned_choice": {k: info[k] for k in ("in_row_bytes", "out_row_bytes", "order_out", "persistent",
                                              "tile_kib", "cache", "fill", "force_ragged")},
        "speedup_batched_call_vs_per_job": round(t_per / t_oneshot, 2),
        "speedup_tuned_graph_vs_per_job": round(t_per / t_tuned, 2),
        "sizes_elems_min_median_max": [int(x) for x in __import__("numpy").percentile(
            [s // e["esize"] for s, e in zip(sizes, specs)], [0, 50, 100])],
    }


def _serve_run(rr, rr_synth, torch, rate, nreq, direct, small_specs, large_specs):
    """Open-loop Poisson arrivals after an untimed warm-up; latency from the
    scheduled arrival to completion."""
    import numpy as np
    budget = 96 << 30
    srv = rr.Server(budget, max_inflight=4, max_batch_jobs=1024, chunk_bytes=64 << 20, tick_us=5,
                    direct=direct, queue_capacity=1 << 20)
    try:
        # resident inputs in the server's budget
        def resident(specs, seed):
            ptrs = []
            for s in specs:
                n = int(np.prod(s["dims"])) * s["esize"]
                p = srv.alloc(n)
                ptrs.append(p)
            return ptrs
        sp = resident(small_specs, 1)
        lp = resident(large_specs, 2)
        small_jobs = rr.make_jobs([(0, p, s["dims"], s["perm"], s["esize"]) for p, s in zip(sp, small_specs)])
        large_jobs = rr.make_jobs([(0, p, s["dims"], s["perm"], s["esize"]) for p, s in zip(lp, large_specs)])
        # warm-up, not timed: every large job and a few hundred small ones, so the
        # kernels' code is loaded and the arena holds slabs before the clock starts
        # (a fresh server otherwise spends its first milliseconds on both)
        lib = rr.lib()
        import ctypes
        tk = ctypes.c_uint64()
        warm = list(large_jobs) + [small_jobs[k] for k in range(0, len(small_jobs), 16)]
        warm_t = set()
        for job in warm:
            rr.check(lib.rr_serve_submit(srv.h, ctypes.byref(job), ctypes.byref(tk)))
            warm_t.add(tk.value)
        while warm_t:
            for t in srv.completions():
                rr.check(srv.poll(t).status)
                srv.release(t)
                warm_t.discard(t)
            time.sleep(0.0002)
        stats0 = srv.stats()
        g = rr_synth.rng(int(rate))
        arrivals = rr_synth.poisson_arrivals(int(rate) + 7, rate, nreq)
        is_large = g.random(nreq) < 0.01
        pick_s = g.integers(0, len(small_specs), nreq)
        pick_l = g.integers(0, len(large_specs), nreq)
        nbytes_small = [int(np.prod(s["dims"])) * s["esize"] for s in small_specs]
        nbytes_large = [int(np.prod(s["dims"])) * s["esize"] for s in large_specs]
        sched = np.empty(nreq, dtype=np.int64)
        lat = {}
        tick_of = {}
        busy = 0
        t0 = time.monotonic_ns() + 2_000_000
        for i in range(nreq):
            ts = t0 + int(arrivals[i] * 1e9)
            sched[i] = ts
            while time.monotonic_ns() < ts:
                pass
            job = large_jobs[pick_l[i]] if is_large[i] else small_jobs[pick_s[i]]
            while True:
                st = lib.rr_serve_submit(srv.h, ctypes.byref(job), ctypes.byref(tk))
                if st != 6:
                    break
                busy += 1
                _drain(srv, lat, tick_of)
            rr.check(st)
            tick_of[tk.value] = i
            if i % 64 == 0:
                _drain(srv, lat, tick_of)
        while len(lat) < nreq:
            _drain(srv, lat, tick_of)
            time.sleep(0.0002)
        t_end = max(v[1] for v in lat.values())
        stats = srv.stats()
    finally:
        srv.close()
    lat_us = np.array([(lat[i][1] - sched[i]) / 1e3 for i in range(nreq)])
    # where the time goes: client lag (scheduled arrival -> submit), submit -> admit
    # (queued for memory or a slot), admit -> launch (waiting to join a batch),
    # launch -> done (on the device, including the wait behind earlier batches)
    parts = {"client_lag": [(lat[i][0] - sched[i]) / 1e3 for i in range(nreq)],
             "submit_to_admit": [(lat[i][2] - lat[i][0]) / 1e3 for i in range(nreq)],
             "admit_to_launch": [(lat[i][3] - lat[i][2]) / 1e3 for i in range(nreq)],
             "launch_to_done": [(lat[i][1] - lat[i][3]) / 1e3 for i in range(nreq)]}
    small_mask = ~is_large
    moved = sum(nbytes_large[pick_l[i]] if is_large[i] else nbytes_small[pick_s[i]] for i in range(nreq))
    span = (t_end - sched[0]) / 1e9
    pct = lambda a, q: round(float(np.percentile(a, q)), 1)
    return {"p50_us": pct(lat_us, 50), "p99_us": pct(lat_us, 99), "p999_us": pct(lat_us, 99.9),
            "small_p50_us": pct(lat_us[small_mask], 50), "small_p99_us": pct(lat_us[small_mask], 99),
            "large_p50_us": pct(lat_us[is_large], 50) if is_large.any() else None,
            "aggregate_GBps": round(2 * moved / span / 1e9, 1), "offered_GBps": round(2 * moved / (arrivals[-1]) / 1e9, 1),
            "requests": nreq, "large_requests": int(is_large.sum()), "batches": stats["batches"] - stats0["batches"],
            "budget_peak_GiB": round(stats["budget_peak"] / 2**30, 2),
            "reserved_peak_GiB": round(stats["reserved"] / 2**30, 2), "busy_retries": busy,
            "breakdown_us": {k: {"p50": pct(np.array(v), 50), "p99": pct(np.array(v), 99)} for k, v in parts.items()}}


def _drain(srv, lat, tick_of):
    for t in srv.completions():
        r = srv.poll(t)
        if r.status != 0:
            raise RuntimeError(f"served job failed with status {r.status}")
        lat[tick_of.pop(t)] = (r.t_submit_ns, r.t_done_ns, r.t_admit_ns, r.t_launch_ns)
        srv.release(t)


SERVE_RATES = (5_000, 20_000, 50_000, 100_000, 200_000, 400_000)
SERVE_P99_BOUNDS_US = (1_000, 5_000)


def _serve_requests(rate, nreq_cap):
    """Requests at one arrival rate: about two seconds of arrivals, 10k..nreq_cap."""
    return int(max(10_000, min(nreq_cap, rate * 2)))


def bench_serve(rr, rr_synth, torch, nreq):
    """Config: Poisson arrivals of batched-workload jobs plus 1% large 1-4 GiB transposes,
    served by the continuous-batching server vs one rr_permute launch per request, over
    a sweep of arrival rates; per mode, the highest rate of the sweep whose p99 latency
    stays within 1 ms and within 5 ms (all requests, and the small requests alone),
    with the aggregate GB/s served there."""
    small_specs = rr_synth.sample_jobs(5_0001, njobs=4096)
    large_specs = rr_synth.large_jobs(5_0002, count=4)
    res = {"large_job_shapes": [(s["dims"], s["perm"], s["esize"]) for s in large_specs],
           "rates_per_s": list(SERVE_RATES)}
    for rate in SERVE_RATES:
        n = _serve_requests(rate, nreq)
        res[f"{rate}_per_s"] = {
            "batched": _serve_run(rr, rr_synth, torch, rate, n, False, small_specs, large_specs),
            "per_request": _serve_run(rr, rr_synth, torch, rate, n, True, small_specs, large_specs),
        }
    best = {}
    for mode in ("batched", "per_request"):
        for key, label in (("p99_us", "all"), ("small_p99_us", "small")):
            for bound in SERVE_P99_BOUNDS_US:
                ok = [r for r in SERVE_RATES if res[f"{r}_per_s"][mode][key] <= bound]
                top = max(ok) if ok else None
                best[f"{mode}_{label}_p99_le_{bound}us"] = (
                    {"rate_per_s": top, "aggregate_GBps": res[f"{top}_per_s"][mode]["aggregate_GBps"],
                     "p99_us": res[f"{top}_per_s"][mode][key]} if top else None)
    res["highest_rate_within_p99"] = best
    # beyond what one launch per request sustains: arrivals at 1M/s (a burst)
    nsat = min(nreq, 20_000)
    res["saturated_1M_per_s"] = {
        "batched": _serve_run(rr, rr_synth, torch, 1_000_000, nsat, False, small_specs, large_specs),
        "per_request": _serve_run(rr, rr_synth, torch, 1_000_000, nsat, True, small_specs, large_specs),
    }
    return res


CPU_SAMPLE = [("3d_512x512x256", (512, 512, 256), (2, 1, 0), 4),
              ("3d_512x512x256", (512, 512, 256), (0, 2, 1), 1),
              ("5d_32^5", (32,) * 5, (4, 2, 0, 3, 1), 2),
              ("2d_16384x16384", (16384, 16384), (1, 0), 1),
              ("4d_64x128x128x64", (64, 128, 128, 64), (0, 3, 1, 2), 2),
              ("3d_512x512x256", (512, 512, 256), (1, 2, 0), 2)]


def _oracle_timed(cases, seed, barrier=None):
    """(start, end, bytes read + written) of oracle permutes of seeded bytes, one
    per case in order (inputs generated before the clock starts)."""
    import numpy as np
    import oracle
    import rr_synth
    xs = [rr_synth.random_bytes(seed + i, int(np.prod(d)) * e) for i, (_, d, p, e) in enumerate(cases)]
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    for x, (_, d, p, e) in zip(xs, cases):
        oracle.permute(x, d, p, e)
    return t0, time.perf_counter(), sum(2 * x.size for x in xs)


def cpu_baseline():
    """The oracle (a single-threaded C loop nest, as it stands) on a bounded sample of
    the benchmark workload: once in one thread, then as one process per host core,
    each running the whole sample from a different starting case, started
    together.  The all-core rate is the reported value.  Uses fork, so call it
    before the process touches the GPU."""
    import multiprocessing as mp
    s0, s1, b1 = _oracle_timed(CPU_SAMPLE, 100)
    t1 = s1 - s0
    # every core this process may run on, up to the host's CPU share for one GPU
    # (OMP_NUM_THREADS, which the GPU hosts set to that share): more processes than
    # the share would only time-slice the same cores
    affinity = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS") or affinity)
    ncores = max(1, min(affinity, share))
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(ncores)
    q = ctx.Queue()

    def work(k):
        r = k % len(CPU_SAMPLE)
        q.put(_oracle_timed(CPU_SAMPLE[r:] + CPU_SAMPLE[:r], 200 + 10 * k, barrier))

    procs = [ctx.Process(target=work, args=(k,)) for k in range(ncores)]
    for pr in procs:
        pr.start()
    res = [q.get(timeout=600) for _ in procs]
    for pr in procs:
        pr.join()
    bn = sum(r[2] for r in res)
    tn = max(r[1] for r in res) - min(r[0] for r in res)
    names = "; ".join(f"{n} {p} e{e}" for n, _, p, e in CPU_SAMPLE)
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(bn / tn / 1e9, 3), "unit": "GB/s", "cores": ncores, "kind": "oracle",
            "host": {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity,
                     "cpu_share_OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")},
            "sample": f"{ncores} processes, each running [{names}] from case k mod 6 "
                      f"({bn / 2 / 2**30:.2f} GiB per side in {tn:.1f} s wall)",
            "single_thread": {"value": round(b1 / t1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                              "sample": f"the 6 cases in sequence ({b1 / 2 / 2**30:.2f} GiB per side, {t1:.1f} s)"}}


if __name__ == "__main__":
    main()
