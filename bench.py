#!/usr/bin/env python3
"""Throughput of the WU-VKLB solver on one MI355X.

One benchmark step = one full solve of the workload: initialization from an
initial state already resident in HBM, then every time step to the end
condition (collision, streaming, moments and the per-step CFL update, one
fused HIP kernel per time step; grids of up to 1024 cells run many steps per
launch in one workgroup). Default workload: the 1D Euler shock tube,
N = 65,536 cells to t = 0.2, FP32 (FP64 reported beside it).

Prints one JSON line: value = cells x time steps / second (Mcell-steps/s) of
the timed solves; roofline = algorithmic bytes of the step kernel (each
population read once and written once, 2 Q p s bytes per cell-step, times
the cells and steps of a launch) over its average launch duration, measured
with HIP events on the solver's stream;
cpu_baseline = the FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2608_04283_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (problem factory, precisions, cpu-baseline sample steps)
    "euler1d_sod": (lambda: I.sod(65536), ("fp32", "fp64"), 3500),
    "sw1d_dambreak": (lambda: I.dam_break(1000, c=0.5, k=0.0), ("fp64",), 600),
    "euler2d_quadrants": (lambda: I.quadrants(2048, seed=0, steps=2000), ("fp32",), 4),
    "mhd1d_briowu": (lambda: I.brio_wu(16384), ("fp32",), 300),
    "mhd2d_orszag_tang": (lambda: I.orszag_tang(1024, steps=1000), ("fp32",), 2),
}
DEFAULT = "euler1d_sod"


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


def profiled_traffic(workload, prec, cells_per_launch):
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
# with: the workload itself (1D), or the size its oracle comparison uses (2D),
# which is then run on the GPU beside the timed solves.
GOLDEN = {
    "euler1d_sod": ("oracle_euler1d_sod_n65536.npz", None),
    "sw1d_dambreak": ("oracle_sw1d_dambreak_d1q2_n1000.npz", None),
    "mhd1d_briowu": ("oracle_mhd1d_briowu_n16384.npz", None),
    "euler2d_quadrants": ("oracle_euler2d_quadrants_n512_s0.npz", lambda: I.quadrants(512, seed=0, steps=2000)),
    "mhd2d_orszag_tang": ("oracle_mhd2d_orszag_tang_n256.npz", lambda: I.orszag_tang(256, steps=1000)),
}


def rel_l1(a, b, small=1e-3):
    """Per field sum|a - b| / sum|b|; fields whose L1 norm is below `small`
    times the largest field's (identically zero ones) are measured against
    the largest field's norm."""
    import numpy as np
    num = np.abs(a - b).sum(axis=1)
    den = np.abs(b).sum(axis=1)
    den = np.where(den <= small * den.max(), den.max(), den)
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


def step_kernel(P, steps):
    """The kernel that advances the workload and the steps one launch takes:
    1D grids of up to 1024 cells (256 for MHD) run up to 1024 steps per
    launch in one workgroup
    (k_run1d_wg, the library's rule for its default options); everything else
    launches k_step1d / k_step2d once per step."""
    if P.dim == 1 and P.cells <= (256 if P.system == "mhd" else 1024):
        return "k_run1d_wg", min(1024, steps)
    return f"k_step{P.dim}d", 1


def time_workload(name, prec, K, W, quick=False):
    import torch
    from paper_2608_04283_amd import vklb

    factory, _, _ = WORKLOADS[name]
    P = factory()
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
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    step_ms = 0.0
    wall0 = time.perf_counter()
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
    wall = time.perf_counter() - wall0
    total_ms = e0.elapsed_time(e1)
    t_end, n_end, done = s.progress()
    U_final, _, _ = s.moments()
    s.close()
    assert n_end == steps and done, (n_end, steps, done)
    cells = P.cells
    cell_steps = cells * steps * K
    value = cell_steps / (total_ms * 1e-3) / 1e6
    step_time_ms = step_ms / (steps * K)
    kernel, spl = step_kernel(P, steps)
    achieved = alg_bytes_per_cell_step(P, prec) * cells / (step_time_ms * 1e-3) / 1e9
    traffic = profiled_traffic(name, prec, cells)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel, "avg_launch_us": round(step_time_ms * spl * 1e3, 3), "steps_per_launch": spl,
            "us_per_step": round(step_time_ms * 1e3, 3),
            "alg_bytes_per_cell_step": alg_bytes_per_cell_step(P, prec), "cells_per_launch": cells}
    err = error_vs_oracle(name, prec, U_final)
    return {"workload": P.name, "value": value, "ms_per_solve": total_ms / K, "steps_per_solve": steps, "error": err,
            "cells": cells, "t_end": t_end, "roofline": roof, "wall_s": wall, "dtype": "f32" if prec == "fp32" else "f64"}


def serving_bench(count, seed=1, budget=None):
    """Batched serving vs plain per-solve launches on a sample of the mixed
    request stream (systems, sizes and step counts drawn as in
    inputs.serving_requests). Capacity = solves/s of the batched pool with
    every request present at once; the timed streams then arrive as a Poisson
    process at 80 % of that capacity, once through the pool and once through
    plain per-solve launches."""
    import torch
    from paper_2608_04283_amd import serving
    if budget is None:
        free, _ = torch.cuda.mem_get_info()
        budget = int(min(free * 0.6, 96 << 30)) // 256 * 256
    reqs = I.serving_requests(count, seed=seed)
    cell_steps = sum(r.problem.cells * r.steps for r in reqs)
    cap = serving.run_batched(reqs, budget, "fp32", realtime=False)
    rate = 0.8 * cap["solves_per_s"]
    timed = serving.with_arrivals(reqs, rate, seed=seed + 1)
    batched = serving.run_batched(timed, budget, "fp32", realtime=True)
    plain_cap = serving.run_plain(reqs, "fp32", realtime=False)
    plain = serving.run_plain(timed, "fp32", realtime=True)
    keep = ("solves", "makespan_s", "solves_per_s", "p50_s", "p99_s", "mcell_steps_per_s", "nonphysical", "failed")
    r = lambda d: {k: (round(d[k], 4) if isinstance(d[k], float) else d[k]) for k in keep}
    return {"requests": count, "seed": seed, "cell_steps": cell_steps, "arena_bytes": budget,
            "capacity_solves_per_s": round(cap["solves_per_s"], 3),
            "capacity_mcell_steps_per_s": round(cap["mcell_steps_per_s"], 1),
            "arrival_rate_per_s": round(rate, 3),
            "batched": r(batched), "plain": r(plain),
            "plain_capacity_solves_per_s": round(plain_cap["solves_per_s"], 3),
            "batched_over_plain_capacity": round(cap["solves_per_s"] / plain_cap["solves_per_s"], 3)}


def cpu_baseline(name):
    from oracle import oracle as O
    factory, _, sample_steps = WORKLOADS[name]
    P = factory()
    kw = dict(system=P.system, dim=P.dim, n=P.n if P.dim == 2 else (P.n[0], 1), lo=P.lo, hi=P.hi, g=P.g,
              gamma=P.gamma, ch_factor=P.ch_factor, adv=P.adv, xi_mode=P.xi_mode, nu=P.nu, xi=P.xi,
              omega=P.omega, c=P.c, k=P.k, bc=P.bc, T=P.T, max_steps=sample_steps)
    cf = O.make_config(**kw)
    t0 = time.perf_counter()
    r = O.run(cf, P.U0)
    dt = time.perf_counter() - t0
    return {"value": round(P.cells * r["steps"] / dt / 1e6, 3), "unit": "Mcell-steps/s", "cores": r["threads"],
            "kind": "oracle",
            "sample": f"first {r['steps']} time steps of {P.name} (FP64 oracle, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed full solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-other-precision", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests in the serving sample (0: skip serving)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (a plain copy kernel of known size, "
                         "for scaling the HBM byte counters) and exit")
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
        nbytes = args.calibrate_copy << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}))
        return
    _, precs, _ = WORKLOADS[args.workload]
    prec = args.precision or precs[0]
    main_res = time_workload(args.workload, prec, args.steps, args.warmup)
    out = {
        # the headline metric; its HBM fraction is roofline.frac, FP64 is under
        # other_precision, served solves/s and p50/p99 latency under serving
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
        "config": {"workload": main_res["workload"], "cells": main_res["cells"],
                   "time_steps_per_solve": main_res["steps_per_solve"], "t_end": main_res["t_end"],
                   "lattice": "D1Q3" if "1d" in args.workload else "D2Q5", "omega": 1.0, "c": 0.05, "k": 2.0},
        "roofline": main_res["roofline"],
        "error_vs_oracle": main_res["error"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    extra = {}
    for p2 in precs:
        if p2 != prec and not args.no_other_precision:
            r = time_workload(args.workload, p2, max(1, args.steps // 2), 1)
            extra[p2] = {"value": round(r["value"], 2), "ms_per_solve": round(r["ms_per_solve"], 4),
                         "roofline": r["roofline"], "error_vs_oracle": r["error"]}
    if extra:
        out["other_precision"] = extra
    if not args.no_also:
        also = {}
        for name, (_, wprecs, _) in WORKLOADS.items():
            if name == args.workload:
                continue
            r = time_workload(name, wprecs[0], 2, 1)
            also[name] = {"value": round(r["value"], 2), "dtype": r["dtype"], "ms_per_solve": round(r["ms_per_solve"], 3),
                          "steps_per_solve": r["steps_per_solve"], "roofline": r["roofline"],
                          "error_vs_oracle": r["error"]}
        out["also"] = also
    if args.serving_requests > 0:
        out["serving"] = serving_bench(args.serving_requests)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
