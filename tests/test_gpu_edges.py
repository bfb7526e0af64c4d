"""Edge sizes on the GPU against the FP64 oracle, element by element.

Grids of one to a few cells (a cell that is its own periodic neighbour, a
zero-gradient ghost that is the only cell), sizes one either side of a 1D
workgroup tile (254 cells), of the one-workgroup limit (1024 cells, MHD 256),
of a 2D strip (256 columns, 64 and 128 for narrow grids) and of a band (32
rows, MHD 8), on both boundary rules, both precisions and both 1D paths (one
workgroup for small grids, one launch per step). Characteristic boundaries
take their smallest grids: two cells, and three, whose middle cell is the
neighbour of both boundaries. Tolerances as in the other parity tests:
relative L1 per field <= 1e-12 (FP64) and <= 1e-4 (FP32).
"""
import numpy as np
import pytest

from paper_2608_04283_amd import inputs as I
from parity_util import rel_l1, run_oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4}


def two_state_2d(system, nx, ny, seed, **kw):
    """Two-state data on an nx x ny grid with dx == dy, the left state on
    x + y < 1, drawn in the ranges of the mixed-request stream."""
    P = I.random_riemann(system, 2, 4, seed, **kw)
    P = P.with_(n=(nx, ny), hi=(nx / ny, 1.0), name=f"{system}2d_two_state_{nx}x{ny}_s{seed}")
    rng = I.SplitMix64(seed)
    sides = []
    for _ in range(2):
        if system == "sw":
            sides.append([rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)])
        else:
            sides.append([rng.uniform(0.5, 1.5), rng.uniform(0.3, 1.5), rng.uniform(-0.5, 0.5),
                          rng.uniform(-0.5, 0.5), rng.uniform(-1.0, 1.0)])
    X, Y = I.grid2(nx, ny, P.lo, P.hi)
    S = np.array(sides)[np.where((X + Y) < 1.0, 0, 1)]
    if system == "sw":
        U0 = I.sw_state(S[..., 0], S[..., 1], S[..., 2])
    elif system == "euler":
        U0 = I.euler_state(S[..., 0], S[..., 2], S[..., 1], P.gamma, v=S[..., 3])
    else:
        z = np.zeros(S.shape[:-1])
        U0 = I.mhd_state(S[..., 0], S[..., 2], S[..., 3], z, S[..., 1], 0.75 + z, S[..., 4], z, P.gamma)
    return P.with_(U0=U0)


def check(gpu, oracle, P, prec, **opts):
    print(f"[edge] {P.name} n={P.n} bc={P.bc} prec={prec} opts={opts}", flush=True)
    ref = run_oracle(oracle, P)
    assert ref["status"] == 0
    s = gpu.Solver(P, precision=prec, **opts)
    s.init()
    U, t, n = s.run()
    s.close()
    assert n == ref["steps"] == P.max_steps
    assert abs(t - ref["t"]) <= (1e-13 if prec == "fp64" else 1e-6) * max(1.0, abs(ref["t"]))
    err = rel_l1(U, ref["U"])
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("path", ["one_workgroup", "launches"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("bc", ["periodic", "zero_gradient"])
@pytest.mark.parametrize("n", [1, 2, 5])
@pytest.mark.parametrize("system", ["sw", "euler", "mhd"])
def test_tiny_1d_grids(gpu, oracle, system, n, bc, prec, path):
    P = I.random_riemann(system, 1, n, 11 + n, max_steps=25, bc=(bc, bc))
    check(gpu, oracle, P, prec, small_grid=0 if path == "one_workgroup" else -1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("path", ["one_workgroup", "launches"])
def test_tiny_1d_grids_characteristic(gpu, oracle, path, n, prec):
    P = I.random_riemann("euler", 1, n, 5, max_steps=25, bc=("characteristic", "characteristic"))
    check(gpu, oracle, P, prec, small_grid=0 if path == "one_workgroup" else -1)


@pytest.mark.parametrize("bc", ["periodic", "zero_gradient"])
@pytest.mark.parametrize("n", [253, 254, 255, 508, 509])
def test_1d_tile_edges(gpu, oracle, n, bc):
    """One launch per step, 254 cells per workgroup tile."""
    P = I.random_riemann("euler", 1, n, 21, max_steps=60, bc=(bc, bc))
    check(gpu, oracle, P, "fp64", small_grid=-1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("system,n", [("euler", 1024), ("euler", 1025), ("mhd", 256), ("mhd", 257)])
def test_1d_one_workgroup_limit(gpu, oracle, system, n, prec):
    """Default options: up to the limit the steps run in one workgroup, past
    it one launch per step."""
    P = I.random_riemann(system, 1, n, 31, max_steps=80)
    check(gpu, oracle, P, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("bc", ["periodic", "zero_gradient"])
@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (5, 1), (2, 3)])
@pytest.mark.parametrize("system", ["sw", "euler", "mhd"])
def test_tiny_2d_grids(gpu, oracle, system, shape, bc, prec):
    P = two_state_2d(system, shape[0], shape[1], 41, max_steps=12, bc=(bc, bc))
    check(gpu, oracle, P, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("system,shape", [
    ("euler", (256, 32)), ("euler", (257, 33)), ("euler", (255, 31)), ("euler", (64, 3)), ("euler", (65, 3)),
    ("euler", (128, 2)), ("euler", (129, 2)), ("mhd", (256, 8)), ("mhd", (257, 9)), ("sw", (257, 65)),
])
def test_2d_strip_and_band_edges(gpu, oracle, system, shape, prec):
    """Strip width and band height at and one past their default sizes, on
    mixed boundary rules (periodic in x, zero gradient in y)."""
    P = two_state_2d(system, shape[0], shape[1], 51, max_steps=20, bc=("periodic", "zero_gradient"))
    check(gpu, oracle, P, prec)


EDGE_PROBLEMS = {
    "euler1d_n1_periodic": (lambda: I.random_riemann("euler", 1, 1, 61, max_steps=20, bc=("periodic", "periodic")), {}),
    "euler1d_n3_characteristic": (lambda: I.random_riemann("euler", 1, 3, 62, max_steps=20,
                                                           bc=("characteristic", "characteristic")), {"small_grid": -1}),
    "mhd1d_n2_zero_gradient": (lambda: I.random_riemann("mhd", 1, 2, 63, max_steps=20), {"small_grid": -1}),
    "mhd2d_1x1_zero_gradient": (lambda: two_state_2d("mhd", 1, 1, 64, max_steps=10), {}),
    "euler2d_2x3_periodic": (lambda: two_state_2d("euler", 2, 3, 65, max_steps=10, bc=("periodic", "periodic")), {}),
    "sw2d_257x33_mixed": (lambda: two_state_2d("sw", 257, 33, 66, max_steps=15, bc=("periodic", "zero_gradient")), {}),
}


@pytest.mark.parametrize("prec,basis", [("fp64", 1), ("fp64", 2), ("fp32", 1), ("fp32", 2), ("fp32", 3)])
@pytest.mark.parametrize("name", list(EDGE_PROBLEMS))
def test_edge_grids_every_basis(gpu, oracle, name, prec, basis):
    """The stored bases (populations, delta, compensated) at edge sizes: the
    delta bases collide halo cells and band edge rows with one population."""
    factory, opts = EDGE_PROBLEMS[name]
    check(gpu, oracle, factory(), prec, basis=basis, **opts)


def test_tiny_grids_served(gpu, oracle):
    """Grids of one to a few cells in the serving pool, every system, both
    dimensions and boundary rules: the same bits as alone, and the oracle's
    result to the FP32 tolerance."""
    probs = []
    for k, system in enumerate(("sw", "euler", "mhd")):
        for n in (1, 2, 5):
            bc = ("periodic", "periodic") if n != 2 else ("zero_gradient", "zero_gradient")
            probs.append(I.random_riemann(system, 1, n, 70 + 3 * k + n, max_steps=15 + n, bc=bc))
        for shape in ((1, 1), (1, 5), (5, 1), (2, 3)):
            bc = ("zero_gradient", "periodic") if shape[0] > shape[1] else ("periodic", "zero_gradient")
            probs.append(two_state_2d(system, shape[0], shape[1], 80 + k, max_steps=9 + shape[1], bc=bc))
    pool = gpu.Pool(1 << 28, "fp32")
    for i, P in enumerate(probs):
        pool.submit(P, tag=i)
    got = {}
    while len(got) < len(probs):
        pool.run(8)
        for c in pool.poll():
            got[c["tag"]] = c
    pool.close()
    for i, P in enumerate(probs):
        print(f"[served] {P.name} n={P.n} bc={P.bc}", flush=True)
        c = got[i]
        s = gpu.Solver(P, precision="fp32")
        s.init()
        U, t, n = s.run()
        s.close()
        assert c["status"] == 0 and c["steps"] == n == P.max_steps and c["t"] == t
        assert np.array_equal(c["U"], U), P.name
        ref = run_oracle(oracle, P)
        assert ref["status"] == 0 and ref["steps"] == n
        assert np.all(rel_l1(U, ref["U"]) <= TOL["fp32"]), P.name
