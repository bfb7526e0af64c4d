"""The Riemann tables of Sec. 5.1 and 5.2 on the HIP path at the finest
lattice each figure of the paper uses (4096 cells for shallow water, 8192
for Sod and the sonic point, 16384 for Leblanc), checked against the exact
Riemann solutions: both precisions run to the end time, FP32 loses no
accuracy against FP64 (the difference is far below the discretization
error), and the error keeps falling from the oracle's value on a lattice
four times coarser.
"""
import numpy as np
import pytest

from exact_riemann import cell_average_exact
from parity_util import run_oracle
from test_oracle_paper_riemann import _exact, _problem

pytestmark = pytest.mark.gpu

FINEST = {"standard": 4096, "hydraulic": 4096, "compression": 4096, "sod": 8192, "sonic": 8192,
          "leblanc": 16384}


def _err(P, which, U, t):
    f, x0, _ = _exact(P, which)
    n = P.n[0]
    e = cell_average_exact(f, np.linspace(P.lo[0], P.hi[0], n + 1), t, x0, sub=2)
    return np.array([np.abs(U[i] - e[i]).mean() for i in range(U.shape[0])])


@pytest.mark.parametrize("which", list(FINEST))
def test_table_problem_at_finest_lattice(gpu, oracle, which):
    n = FINEST[which]
    P = _problem(which, n)
    print(f"[case] {which} n={n}", flush=True)
    errs = {}
    for prec in ("fp64", "fp32"):
        s = gpu.Solver(P, precision=prec)
        s.init()
        U, t, steps = s.run()
        s.close()
        assert abs(t - P.T) <= 1e-6 * P.T
        assert np.all(np.isfinite(U))
        errs[prec] = _err(P, which, U, t)
    coarse = _problem(which, n // 4)
    r = run_oracle(oracle, coarse)
    e_coarse = _err(coarse, which, r["U"], r["t"])
    print(f"[case] {which} L1 fp64={errs['fp64']} fp32={errs['fp32']} oracle(n/4)={e_coarse}", flush=True)
    assert np.all(np.abs(errs["fp32"] - errs["fp64"]) <= 0.01 * errs["fp64"]), errs
    assert np.all(errs["fp64"] < 0.6 * e_coarse), (errs["fp64"], e_coarse)
