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
from parity_util import oracle_config  # noqa: E402

GOLDENS = {
    # name: (problem factory, storage dtype)
    "sw1d_dambreak_d1q2_n1000": (lambda: I.dam_break(1000, c=0.5, k=0.0), np.float64),
    "sw1d_dambreak_wu_n1000_100steps": (lambda: I.dam_break(1000, max_steps=100), np.float64),
    "euler1d_sod_n65536": (lambda: I.sod(65536), np.float64),
    "euler1d_wave_n256": (lambda: I.smooth_wave(256), np.float64),
    "euler1d_wave_n1024": (lambda: I.smooth_wave(1024), np.float64),
    "euler1d_wave_n4096": (lambda: I.smooth_wave(4096), np.float64),
    "euler2d_quadrants_n512_s0": (lambda: I.quadrants(512, seed=0, steps=2000), np.float32),
    "mhd2d_orszag_tang_n256": (lambda: I.orszag_tang(256, steps=1000), np.float32),
    "mhd1d_briowu_n16384": (lambda: I.brio_wu(16384), np.float32),
}


def oracle_sha():
    return hashlib.sha256(open(os.path.join(ROOT, "oracle", "vklb_oracle.cpp"), "rb").read()).hexdigest()[:16]


def main(names):
    O.build()
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
    main(sys.argv[1:] or list(GOLDENS))
