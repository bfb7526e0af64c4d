"""The C ABI alone, from a plain C99 program (tests/c/abi_run.c) with no
Python or torch in its process: it creates a solver that allocates its own
workspace, runs a Sod shock tube to its end time and reads U back; the result
matches the oracle to the path's tolerance."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2608_04283_amd import inputs as I
from parity_util import rel_l1, run_oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = {"fp64": 1e-12, "fp32": 1e-4}


@pytest.fixture(scope="module")
def abi_run(tmp_path_factory, gpu):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lib_dir = os.path.dirname(gpu.LIB_PATH)
    exe = str(tmp_path_factory.mktemp("cabi") / "abi_run")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_run.c"), "-L", lib_dir, "-lvklb", "-Wl,-rpath," + lib_dir,
                    "-lm", "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c_program_runs_the_step(abi_run, oracle, prec):
    n, T = 3000, 0.05
    print(f"[case] C ABI Sod n={n} T={T} {prec}", flush=True)
    r = subprocess.run([abi_run, str(n), repr(T), prec], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    t, steps = lines[0].split()
    U = np.array([float(v) for v in lines[1:1 + 3 * n]]).reshape(3, n)
    ref = run_oracle(oracle, I.sod(n, T=T))
    assert float(t) == pytest.approx(T, abs=1e-13)
    assert abs(int(steps) - ref["steps"]) <= (0 if prec == "fp64" else 1)
    err = rel_l1(U, ref["U"])
    print(f"[case] steps={steps} rel_l1={err}", flush=True)
    assert np.all(err <= TOL[prec]), err
