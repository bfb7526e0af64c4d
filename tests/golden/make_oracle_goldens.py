"""Write the oracle's full-length results for the benchmark configurations
(tests/golden/oracle_*.npz). Calls only oracle/ and the seeded input
generators; the GPU tests compare the HIP path against these files.

FP32 configurations are stored rounded to float32 (the comparison tolerance,
1e-4 relative L1, is far above that rounding); FP64 ones in float64.
"""
import hashlib
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from oracle import oracle as O  # noqa: E402
from paper_2608_04283_amd import inputs as I  # noqa: E402
from parity_util import oracle_config, serving_sample  # noqa: E402

GOLDENS = {
    # name: (problem factory, storage dtype)
    "sw1d_dambreak_d1q2_n1000": (lambda: I.dam_break(1000, c=0.5, k=0.0), np.float64),
    "sw1d_dambreak_wu_n1000": (lambda: I.dam_break(1000), np.float64),
    "euler1d_sod_n65536": (lambda: I.sod(65536), np.float64),
    "euler1d_wave_n256": (lambda: I.smooth_wave(256), np.float64),
    "euler1d_wave_n1024": (lambda: I.smooth_wave(1024), np.float64),
    "euler1d_wave_n4096": (lambda: I.smooth_wave(4096), np.float64),
    "euler1d_wave_n16384": (lambda: I.smooth_wave(16384), np.float64),
    "euler2d_quadrants_n512_s0": (lambda: I.quadrants(512, seed=0, steps=2000), np.float32),
    "mhd2d_orszag_tang_n256": (lambda: I.orszag_tang(256, steps=1000), np.float32),
    "mhd1d_briowu_n16384": (lambda: I.brio_wu(16384), np.float32),
}


def oracle_sha():
    return hashlib.sha256(open(os.path.join(ROOT, "oracle", "vklb_oracle.cpp"), "rb").read()).hexdigest()[:16]


def write_serving():
    """oracle_serving_seed1.npz: per request (by rid) U (float32), t, steps,
    status, fail step and cell of the FP64 oracle run of the materialized
    request (FP32 requests in the pool; tolerance 1e-4)."""
    out = {}
    for r in serving_sample():
        P = I.materialize(r.problem)
        t0 = time.time()
        res = O.run(oracle_config(O, P), P.U0)
        out[f"U_{r.rid}"] = res["U"].astype(np.float32)
        out[f"meta_{r.rid}"] = np.array([res["t"], res["steps"], res["status"], res["fail_step"], res["fail_cell"]],
                                        dtype=np.float64)
        print(f"serving rid={r.rid} {P.name}: steps={res['steps']} status={res['status']} "
              f"fail=({res['fail_step']},{res['fail_cell']}) {time.time() - t0:.0f}s", flush=True)
    path = os.path.join(HERE, "oracle_serving_seed1.npz")
    np.savez_compressed(path, rids=np.array(sorted(int(k[2:]) for k in out if k.startswith("U_"))),
                        oracle_sha=oracle_sha(), **out)
    print(f"serving: {os.path.getsize(path) / 1e6:.2f} MB", flush=True)


def serving_spread(rel=1e-7, seeds=(1, 2)):
    """Adds spread_<rid> to oracle_serving_seed1.npz for the 1D requests: the
    largest relative L1 per field between the stored run and runs from the
    initial state perturbed by `rel` (the order of FP32 rounding) times a
    standard normal per value. At the 1D CFL number 0.9 the weighted split
    amplifies rounding near slow states, and a request whose spread is large
    has no answer unique to that precision. The 2D requests run at CFL 0.4,
    inside the split's linear stability bound, and get no entry."""
    path = os.path.join(HERE, "oracle_serving_seed1.npz")
    data = dict(np.load(path))
    sample = {r.rid: r for r in serving_sample()}
    for rid in data["rids"]:
        r = sample[int(rid)]
        P = I.materialize(r.problem)
        if P.dim != 1 or int(data[f"meta_{rid}"][2]) != 0:
            continue
        ref = O.run(oracle_config(O, P), P.U0)["U"]
        worst = 0.0
        for sd in seeds:
            g = np.random.default_rng(sd).standard_normal(P.U0.shape)
            U = O.run(oracle_config(O, P), P.U0 * (1.0 + rel * g))["U"]
            num = np.abs(U - ref).sum(axis=1)
            den = np.abs(ref).sum(axis=1)
            den = np.where(den <= 1e-12 * den.max(), den.max(), den)
            worst = max(worst, float((num / den).max()))
        data[f"spread_{rid}"] = np.array(worst)
        print(f"serving rid={rid} {P.name}: spread {worst:.2e}", flush=True)
    np.savez_compressed(path, **data)


def main(names):
    O.build()
    if "serving" in names:
        write_serving()
        serving_spread()
        names = [n for n in names if n != "serving"]
    if "serving_spread" in names:
        serving_spread()
        names = [n for n in names if n != "serving_spread"]
    for name in names:
        factory, dt = GOLDENS[name]
        P = factory()
        t0 = time.time()
        r = O.run(oracle_config(O, P), P.U0)
        el = time.time() - t0
        path = os.path.join(HERE, f"oracle_{name}.npz")
        np.savez_compressed(path, U=r["U"].astype(dt), t=r["t"], steps=r["steps"], status=r["status"],
                            totals=r["totals"], oracle_sha=oracle_sha(),
                            u0_sha=hashlib.sha256(np.ascontiguousarray(P.U0).tobytes()).hexdigest()[:16])
        print(f"{name}: steps={r['steps']} t={r['t']} status={r['status']} {el:.0f}s "
              f"{os.path.getsize(path) / 1e6:.2f} MB", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(GOLDENS) + ["serving"])
