"""Serving pool (vklb_pool_*) on the GPU: every solve gives the same bits
alone and in the batch, admission respects the HBM budget, results match the
oracle, failures are reported per request."""
import numpy as np
import pytest

from paper_2608_04283_amd import inputs as I
from paper_2608_04283_amd import serving
from parity_util import rel_l1, run_oracle

pytestmark = pytest.mark.gpu


def small_mix(count, seed):
    rng = I.SplitMix64(seed)
    out = []
    for rid in range(count):
        system = ("sw", "euler", "mhd")[rid % 3]
        dim = 1 + (rid // 3) % 2
        n = rng.randint(300, 3000) if dim == 1 else rng.randint(40, 160)
        steps = rng.randint(20, 120)
        P = I.random_riemann(system, dim, n, seed=seed * 1000 + rid, max_steps=steps)
        out.append(I.Request(rid=rid, arrival=0.0, problem=P, steps=steps))
    return out


def alone(gpu, P):
    s = gpu.Solver(P, precision="fp32")
    s.init()
    U, t, n = s.run()
    s.close()
    return U, t, n


def test_alone_equals_mix_bitwise(gpu):
    reqs = small_mix(18, seed=4)
    pool = gpu.Pool(2 << 30, "fp32")
    for rq in reqs:
        pool.submit(rq.problem, tag=rq.rid)
    got = {}
    while len(got) < len(reqs):
        pool.run(16)
        for c in pool.poll():
            got[c["tag"]] = c
    pool.close()
    for rq in reqs:
        c = got[rq.rid]
        U, t, n = alone(gpu, rq.problem)
        assert c["status"] == 0 and c["steps"] == n == rq.steps
        assert c["t"] == t
        assert np.array_equal(c["U"], U), rq.problem.name


def test_characteristic_boundaries_served_bitwise(gpu):
    """1D solves with characteristic boundaries (every system, grids in one
    workgroup and above, and the three- and two-cell grids whose middle or
    other cell is the neighbour of both boundaries) give the same bits served
    by the pool, next to periodic ones, as alone."""
    reqs = []
    for rid, (system, n, steps) in enumerate((("sw", 700, 60), ("euler", 1500, 90), ("mhd", 200, 40),
                                              ("mhd", 2100, 50), ("euler", 600, 30), ("sw", 3000, 70),
                                              ("euler", 3, 25), ("mhd", 3, 25), ("sw", 2, 25))):
        P = I.random_riemann(system, 1, n, seed=900 + rid, max_steps=steps)
        if rid != 4:
            P = P.with_(bc=("characteristic", "characteristic"))
        reqs.append(I.Request(rid=rid, arrival=0.0, problem=P, steps=steps))
    pool = gpu.Pool(1 << 30, "fp32")
    for rq in reqs:
        pool.submit(rq.problem, tag=rq.rid)
    got = {}
    while len(got) < len(reqs):
        pool.run(8)
        for c in pool.poll():
            got[c["tag"]] = c
    pool.close()
    for rq in reqs:
        c = got[rq.rid]
        U, t, n = alone(gpu, rq.problem)
        assert c["status"] == 0 and c["steps"] == n == rq.steps and c["t"] == t
        assert np.array_equal(c["U"], U), rq.problem.name


def test_admission_under_small_budget(gpu):
    reqs = small_mix(9, seed=5)
    sizes = [gpu.workspace_bytes(r.problem, "fp32") for r in reqs]
    budget = (max(sizes) * 2 + (1 << 20)) // 256 * 256 + (1 << 20)
    pool = gpu.Pool(budget, "fp32")
    for rq in reqs:
        pool.submit(rq.problem, tag=rq.rid)
    pool.run(0)
    st = pool.stats()
    assert st["queued"] > 0 and st["resident"] >= 1
    got = {}
    while len(got) < len(reqs):
        pool.run(8)
        for c in pool.poll():
            got[c["tag"]] = c
    st = pool.stats()
    pool.close()
    assert st["arena_peak"] <= budget
    assert st["completed"] == len(reqs) and st["resident"] == 0 and st["queued"] == 0
    for rq in reqs[:4]:
        U, _, _ = alone(gpu, rq.problem)
        assert np.array_equal(got[rq.rid]["U"], U)


def test_pool_results_match_oracle(gpu, oracle):
    reqs = small_mix(6, seed=6)
    pool = gpu.Pool(1 << 30, "fp32")
    for rq in reqs:
        pool.submit(rq.problem, tag=rq.rid)
    got = {}
    while len(got) < len(reqs):
        pool.run(32)
        for c in pool.poll():
            got[c["tag"]] = c
    pool.close()
    for rq in reqs:
        ref = run_oracle(oracle, rq.problem)
        err = rel_l1(got[rq.rid]["U"], ref["U"])
        print(rq.problem.name, err.max())
        assert np.all(err <= 1e-4), (rq.problem.name, err)


def test_request_larger_than_arena_rejected(gpu):
    pool = gpu.Pool(4 << 20, "fp32")
    big = I.quadrants(512, steps=10)
    with pytest.raises(gpu.VklbError) as ei:
        pool.submit(big)
    assert ei.value.status == gpu.ERR_OOM
    pool.close()


def test_nonphysical_request_reported(gpu, oracle):
    bad = I.sod(200, omega=1.95, T=float("inf"), max_steps=5000)
    ok = I.sod(300, max_steps=100)
    ref = run_oracle(oracle, bad)
    pool = gpu.Pool(1 << 28, "fp64")
    pool.submit(bad, tag=1)
    pool.submit(ok, tag=2)
    got = {}
    while len(got) < 2:
        pool.run(64)
        for c in pool.poll():
            got[c["tag"]] = c
    pool.close()
    assert got[1]["status"] == gpu.ERR_NONPHYSICAL
    assert got[1]["fail_step"] == ref["fail_step"] and got[1]["fail_cell"] == ref["fail_cell"]
    assert got[2]["status"] == 0 and got[2]["steps"] == 100


def test_request_loop_latencies(gpu):
    reqs = serving.with_arrivals(small_mix(10, seed=7), rate=40.0)
    res = serving.run_batched(reqs, 1 << 30, "fp32", chunk_rounds=16)
    assert res["solves"] == 10 and res["nonphysical"] == 0
    assert 0.0 < res["p50_s"] <= res["p99_s"]
    plain = serving.run_plain(reqs[:3], "fp32")
    assert plain["solves"] == 3 and plain["p50_s"] > 0
