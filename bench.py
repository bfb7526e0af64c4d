#!/usr/bin/env python3
"""Throughput of the WU-VKLB solver on one MI355X.

One benchmark step = one full solve of the workload: initialization from an
initial state already resident in HBM, then every time step to the end
condition (collision, streaming, moments and the per-step CFL update, one
fused HIP kernel per time step; grids of up to 1024 cells run many steps per
launch in one workgroup).

Headline workload: 2D Euler four-quadrant Riemann data, 2048^2 cells, 2000
steps, FP32 populations: the largest single-GPU configuration, and the one
whose working set (671 MB) is far above the 256 MB Infinity Cache, so its
HBM fraction measures HBM. The other configurations run beside it under
"also" (1D shallow water in both lattice forms, 1D Euler shock tube FP32 and
FP64, the 1D smooth wave to 65,536 cells, 1D and 2D MHD), and the mixed
request stream under "serving".

Prints one JSON line: value = cells x time steps / second (Mcell-steps/s) of
the timed solves; roofline = algorithmic bytes of the step kernel (each
population read once and written once, 2 Q p s bytes per cell-step, times
the cells and steps of a launch) over its average launch duration, measured
with HIP events on the solver's stream; cpu_baseline = the FP64 oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
for _p in (ROOT, os.path.join(ROOT, "tests")):
    if _p not in sys.path:
        sys.path.insert(0, _p)

from paper_2608_04283_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0

# name: problem factory, precisions (first = the one reported first), warm-up
# and timed solves for a line under "also", the oracle window of its CPU
# baseline (time steps), and the lattice it runs (D1Q2 = the weighted set
# with c = 1/2, k = 0, whose rest population is identically zero)
WORKLOADS = {
    "euler2d_quadrants": (lambda: I.quadrants(2048, seed=0, steps=2000), ("fp32",), (1, 3), 20, "D2Q5"),
    "euler1d_sod": (lambda: I.sod(65536), ("fp32", "fp64"), (1, 2), 200, "D1Q3"),
    "euler1d_wave": (lambda: I.smooth_wave(65536), ("fp64", "fp32"), (1, 1), 200, "D1Q3"),
    "sw1d_dambreak": (lambda: I.dam_break(1000), ("fp64",), (1, 3), None, "D1Q3"),
    "sw1d_dambreak_d1q2": (lambda: I.dam_break(1000, c=0.5, k=0.0), ("fp64",), (1, 3), None, "D1Q2"),
    "mhd1d_briowu": (lambda: I.brio_wu(16384), ("fp32",), (1, 2), 400, "D1Q3"),
    "mhd2d_orszag_tang": (lambda: I.orszag_tang(1024, steps=1000), ("fp32",), (1, 3), 10, "D2Q5"),
}
HEADLINE = "euler2d_quadrants"


def log(msg):
    """Progress of the run, on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes_per_cell_step(P, prec):
    return 2 * P.Q * P.p * (4 if prec == "fp32" else 8)


# Files that define the step kernels and their launch parameters (tile
# shapes, bands, halo batches): a change to any of them makes earlier byte
# counts stale. The runtime, the pool and the host cell check are not among
# them.
KERNEL_SOURCES = ("vklb_cell.hpp", "vklb_kernels.hpp", "vklb_launch.hpp", "vklb_host.hpp", "vklb_system.inc",
                  "k_sw.hip", "k_euler.hip", "k_mhd.hip", "k_linear.hip")


def kernel_sources_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2608_04283_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(workload, prec):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_sources_sha:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_sources_sha():
        return None
    return float(b.group(1))


# Stored FP64 oracle results (written by tests/golden/make_oracle_goldens.py,
# which runs the oracle alone) that each workload's final state is compared
# with: the workload itself, or the size its oracle comparison uses, which is
# then run on the GPU beside the timed solves.
GOLDEN = {
    "euler1d_sod": ("oracle_euler1d_sod_n65536.npz", None),
    "euler1d_wave": ("oracle_euler1d_wave_n16384.npz", lambda: I.smooth_wave(16384)),
    "sw1d_dambreak": ("oracle_sw1d_dambreak_wu_n1000.npz", None),
    "sw1d_dambreak_d1q2": ("oracle_sw1d_dambreak_d1q2_n1000.npz", None),
    "mhd1d_briowu": ("oracle_mhd1d_briowu_n16384.npz", None),
    "euler2d_quadrants": ("oracle_euler2d_quadrants_n512_s0.npz", lambda: I.quadrants(512, seed=0, steps=2000)),
    "mhd2d_orszag_tang": ("oracle_mhd2d_orszag_tang_n256.npz", lambda: I.orszag_tang(256, steps=1000)),
}


def rel_l1(a, b, zero=1e-12):
    """Per field sum|a - b| / sum|b| (b the oracle); a field that is
    identically zero in b (L1 norm at most `zero` times the largest field's)
    is measured against the largest field's norm."""
    import numpy as np
    num = np.abs(a - b).sum(axis=1)
    den = np.abs(b).sum(axis=1)
    den = np.where(den <= zero * den.max(), den.max(), den)
    return num / den


def error_vs_oracle(name, prec, U_final):
    """Relative L1 per field of the final state against the stored oracle run."""
    import numpy as np
    from paper_2608_04283_amd import vklb
    fname, small = GOLDEN[name]
    path = os.path.join(ROOT, "tests", "golden", fname)
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    U, size = U_final, None
    if small is not None:
        P = small()
        s = vklb.Solver(P, precision=prec)
        s.init()
        U, _, _ = s.run()
        s.close()
        size = "x".join(str(v) for v in P.n)
    err = rel_l1(U, ref["U"])
    return {"rel_l1_per_field": [float(f"{e:.3g}") for e in err], "max": float(f"{err.max():.3g}"),
            "at_size": size or "the workload's", "oracle": "FP64"}


def error_vs_exact(name, P, U, t):
    """Mean absolute error of the first field(s) against the exact solution,
    where one exists: the dam break (exact Riemann solution, h and hu) and
    the smooth wave (rho(x - t), exact cell averages)."""
    import numpy as np
    n = P.n[0]
    if name.startswith("sw1d_dambreak"):
        from exact_riemann import ShallowWaterRiemann, cell_average_exact
        ex = ShallowWaterRiemann(2.0, 0.0, 1.0, 0.0, P.g)
        hu = cell_average_exact(lambda s: np.stack(ex.sample(s)), np.linspace(0, 1, n + 1), t, 0.5, sub=4)
        exact = np.stack([hu[0], hu[0] * hu[1]])
        l1 = np.abs(U - exact).mean(axis=1)
        return {"l1_h": float(f"{l1[0]:.4g}"), "l1_hu": float(f"{l1[1]:.4g}"), "exact": "dam-break Riemann solution"}
    if name == "euler1d_wave":
        x = (np.arange(n) + 0.5) / n
        dx = 1.0 / n
        avg = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - dx / 2 - t)) - np.cos(2 * np.pi * (x + dx / 2 - t))) / (2 * np.pi * dx)
        return {"l1_rho": float(f"{np.abs(U[0] - avg).mean():.4g}"), "exact": "rho(x - t) cell averages"}
    return None


def step_kernel(P, steps):
    """The kernel that advances the workload and the steps one launch takes:
    1D grids of up to 1024 cells (256 for MHD) run up to 1024 steps per
    launch in one workgroup (k_run1d_wg, the library's rule for its default
    options); everything else launches k_step1d / k_step2d once per step."""
    if P.dim == 1 and P.cells <= (256 if P.system == "mhd" else 1024):
        return "k_run1d_wg", min(1024, steps)
    return f"k_step{P.dim}d", 1


def time_workload(name, prec, K, W):
    import torch
    from paper_2608_04283_amd import vklb

    P = WORKLOADS[name][0]()
    s = vklb.Solver(P, precision=prec)
    U0 = torch.from_numpy(P.U0).to("cuda").contiguous()
    stream = torch.cuda.current_stream()
    # warm-up solves; the first also fixes the number of time steps of a solve
    steps = None
    for _ in range(max(1, W)):
        s.init_device(U0.data_ptr())
        U, t, n = s.run()
        steps = n
    torch.cuda.synchronize()
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    step_ms = 0.0
    e0.record(stream)
    for k in range(K):
        s.init_device(U0.data_ptr())
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.step(steps)
        b.record(stream)
        if k == K - 1:
            e1.record(stream)
        torch.cuda.synchronize()
        step_ms += a.elapsed_time(b)
    e1.synchronize()
    total_ms = e0.elapsed_time(e1)
    t_end, n_end, done = s.progress()
    U_final, _, _ = s.moments()
    diag = s.diagnostics()
    s.close()
    assert n_end == steps and done, (n_end, steps, done)
    cells = P.cells
    value = cells * steps * K / (total_ms * 1e-3) / 1e6
    step_time_ms = step_ms / (steps * K)
    kernel, spl = step_kernel(P, steps)
    abytes = alg_bytes_per_cell_step(P, prec)
    achieved = abytes * cells / (step_time_ms * 1e-3) / 1e9
    two_d = P.dim == 2
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(name, prec),
            "kernel": kernel, "avg_launch_us": round(step_time_ms * spl * 1e3, 3), "steps_per_launch": spl,
            "us_per_step": round(step_time_ms * 1e3, 3), "alg_bytes_per_cell_step": abytes,
            "cells_per_launch": cells, "populations_mb": round(abytes * cells / 1e6, 1)}
    if not two_d:
        roof["note"] = ("working set cache-resident between steps: the step is bound by the latency of one "
                        "dependent launch, not by HBM")
    out = {"workload": P.name, "value": value, "ms_per_solve": total_ms / K, "steps_per_solve": steps,
           "error": error_vs_oracle(name, prec, U_final), "exact": error_vs_exact(name, P, U_final, t_end),
           "cells": cells, "t_end": t_end, "roofline": roof, "dtype": "f32" if prec == "fp32" else "f64",
           "params": {"lattice": WORKLOADS[name][4], "omega": P.omega, "c": P.c, "k": P.k, "nu": P.nu,
                      "bc": P.bc[0]}}
    if P.system == "mhd" and two_d:
        out["max_div_b"] = float(f"{diag['max_div_b']:.4g}")
    log(f"{P.name} {prec}: {value:.1f} Mcell-steps/s, {step_time_ms * 1e3:.2f} us per step")
    return out


def serving_bench(count, seed=1, budget=None, sample_every=5):
    """Batched serving against plain per-solve launches on the mixed request
    stream (systems, sizes and step counts drawn as in
    inputs.serving_requests, seed 1). Capacity = solves/s of the batched pool
    with every request present at once; the timed stream then arrives as a
    Poisson process at 80 % of that capacity. The plain baseline (one solve
    at a time, the single-solve path with its 512-step graph chunks) is
    measured closed-loop, on every `sample_every`-th request beside the pool
    on the same sample: at the batched arrival rate it cannot keep up, so its
    timed run would only grow its queue. Solves that turn non-physical are
    counted apart from the served solves/s."""
    import torch
    from paper_2608_04283_amd import serving
    if budget is None:
        free, _ = torch.cuda.mem_get_info()
        budget = int(min(free * 0.6, 96 << 30)) // 256 * 256
    t0 = time.perf_counter()
    tiles = serving.tune_shapes("fp32")
    tune_s = time.perf_counter() - t0
    reqs = I.serving_requests(count, seed=seed)
    cell_steps = sum(r.problem.cells * r.steps for r in reqs)
    keep = ("solves", "ok", "nonphysical", "makespan_s", "solves_per_s", "completed_per_s", "p50_s", "p99_s",
            "mcell_steps_per_s", "alg_gb_per_s", "hbm_frac", "graph_launches", "graph_captures")

    def r(d):
        # the stream's aggregate algorithmic bytes (2 Q p s per cell-step of
        # every completed solve) over the makespan, as a fraction of 8 TB/s
        d = dict(d, hbm_frac=d["alg_gb_per_s"] / 8000.0)
        return {k: (round(d[k], 4) if isinstance(d[k], float) else d[k]) for k in keep if k in d}
    log(f"serving: 2D tile shapes tuned in {tune_s:.1f} s")
    prog = lambda what: (lambda k, n: log(f"serving {what}: {k} of {n} solves done"))
    cap = serving.run_batched(reqs, budget, "fp32", realtime=False, progress=prog("capacity"))
    rate = 0.8 * cap["solves_per_s"]
    timed = serving.with_arrivals(reqs, rate, seed=seed + 1)
    batched = serving.run_batched(timed, budget, "fp32", realtime=True, progress=prog("at 80 %"))
    sample = reqs[::sample_every]
    cap_s = serving.run_batched(sample, budget, "fp32", realtime=False)
    log("serving: batched sample done")
    plain_s = serving.run_plain(sample, "fp32", realtime=False, progress=prog("plain sample"))
    names = {0: "sw", 1: "euler", 2: "mhd"}
    return {"requests": count, "seed": seed, "cell_steps": cell_steps, "arena_bytes": budget,
            "tiles_2d": {"tuning_s": round(tune_s, 2),
                         "band_halo": {f"{names[t['kind']]}_{t['n']}": [t["band_rows"], t["halo_rows"]]
                                       for t in tiles}},
            "capacity": r(cap), "arrival_rate_per_s": round(rate, 3), "batched_at_80pct": r(batched),
            "nonphysical_rids": [f[0] for f in cap["failed"]],
            "vs_plain": {"sample": f"every {sample_every}th request ({len(sample)})", "batched": r(cap_s),
                         "plain": r(plain_s),
                         "batched_over_plain_solves_per_s": round(cap_s["solves_per_s"] / plain_s["solves_per_s"], 3),
                         "plain_at_80pct_of_batched_capacity": "overloaded: its capacity is below the arrival rate"
                         if plain_s["solves_per_s"] < rate else "keeps up"}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads():
    """Threads the oracle runs with: OMP_NUM_THREADS when set (the host's
    share of cores), else every core the OS reports."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)


def cpu_baseline(name, steps, threads=None):
    """The FP64 oracle, as it stands, on the first `steps` time steps of the
    workload (threads: host_threads() unless given)."""
    from oracle import oracle as O
    from parity_util import oracle_config
    P = WORKLOADS[name][0]()
    threads = threads or host_threads()
    cf = oracle_config(O, P, threads=threads, max_steps=min(P.max_steps, steps) if steps else P.max_steps)
    t0 = time.perf_counter()
    r = O.run(cf, P.U0)
    dt = time.perf_counter() - t0
    log(f"oracle on {P.name}: {r['steps']} steps, {threads} threads, {dt:.1f} s")
    return {"value": round(P.cells * r["steps"] / dt / 1e6, 3), "unit": "Mcell-steps/s", "cores": r["threads"],
            "kind": "oracle",
            "sample": f"first {r['steps']} time steps of {P.name} (FP64 oracle, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed full solves of the headline workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true", help="skip the other workloads")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the serving stream (0: skip serving)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run the library's streaming copy kernel over MIB MiB (three timed copies) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X (no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy > 0:
        from paper_2608_04283_amd import vklb
        print(json.dumps(vklb.stream_copy_bench(args.calibrate_copy << 20)))
        return
    _, precs, _, cpu_steps, _ = WORKLOADS[args.workload]
    prec = args.precision or precs[0]
    main_res = time_workload(args.workload, prec, args.steps, args.warmup)
    # the copy ceiling beside it: the library's streaming copy (every byte read
    # and written once, one 16-byte word per lane) over 1 GiB
    from paper_2608_04283_amd import vklb
    copy = vklb.stream_copy_bench(1 << 30)["non_temporal"]
    main_res["roofline"]["copy_ceiling"] = {"gb_per_s": copy["gb_per_s"], "bytes": 2 << 30,
                                            "achieved_over_copy": round(main_res["roofline"]["achieved"] /
                                                                        copy["gb_per_s"], 4)}
    log(f"copy ceiling {copy['gb_per_s']:.1f} GB/s")
    out = {
        # the headline metric; its HBM fraction is roofline.frac, the other
        # workloads (FP64 beside FP32) under also, served solves/s with p50/p99
        # latency under serving
        "metric": "Mcell-steps/s & % HBM roofline, FP32 vs FP64; served solves/s, p50/p99 latency",
        "value": round(main_res["value"], 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_solve"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_res["dtype"],
        "data": "synthetic",
        "config": dict({"workload": main_res["workload"], "cells": main_res["cells"],
                        "time_steps_per_solve": main_res["steps_per_solve"], "t_end": main_res["t_end"]},
                       **main_res["params"]),
        "roofline": main_res["roofline"],
        "error_vs_oracle": main_res["error"],
    }
    if main_res.get("exact"):
        out["error_vs_exact"] = main_res["exact"]
    if "max_div_b" in main_res:
        out["max_div_b"] = main_res["max_div_b"]
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.workload, cpu_steps)
        cb["cpu_model"] = cpu_model()
        one = cpu_baseline(args.workload, max(1, (cpu_steps or 20) // 10), threads=1)
        cb["single_thread"] = {"value": one["value"], "sample": one["sample"]}
        out["cpu_baseline"] = cb
    if not args.no_also:
        also = {}
        for name, (_, wprecs, (w, k), csteps, _) in WORKLOADS.items():
            for p2 in wprecs:
                if name == args.workload and p2 == prec:
                    continue
                r = time_workload(name, p2, k, w)
                entry = {"workload": r["workload"], "value": round(r["value"], 2), "dtype": r["dtype"],
                         "ms_per_solve": round(r["ms_per_solve"], 3), "steps_per_solve": r["steps_per_solve"],
                         "params": r["params"], "roofline": r["roofline"], "error_vs_oracle": r["error"]}
                if r.get("exact"):
                    entry["error_vs_exact"] = r["exact"]
                if "max_div_b" in r:
                    entry["max_div_b"] = r["max_div_b"]
                if p2 == wprecs[0] and not args.no_cpu_baseline and name != args.workload:
                    entry["cpu_baseline"] = cpu_baseline(name, csteps)
                also[f"{name}_{p2}"] = entry
        out["also"] = also
    if args.serving_requests > 0:
        out["serving"] = serving_bench(args.serving_requests)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
