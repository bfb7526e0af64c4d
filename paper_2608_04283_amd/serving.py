"""Request loop over the serving pool (vklb_pool_*) and the plain baseline.

Batched serving: requests are submitted to the pool at their arrival times;
between chunks of rounds the pool admits what fits in its HBM arena (the
others wait in order), advances every resident solve, and hands back the
finished ones. Latency = completion time - arrival time, on the host clock.
The pool's 2D tile shapes come from tune_shapes when it ran in the process.

Plain baseline: the single-solve path, one solve at a time in arrival order
(the same kernels, launched as vklb_step launches them: in captured graphs of
512 steps).

Both report every completed request (solves) and, apart, those that ended in
a non-physical state; solves_per_s counts the served (physical) solves only.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time

import numpy as np

from . import inputs
from . import vklb


def _percentiles(lat):
    if not lat:
        return None, None
    a = np.sort(np.asarray(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


class _Prefetch:
    """Builds the initial states of upcoming requests on worker threads."""

    def __init__(self, requests, window=48, workers=4):
        self.reqs = list(requests)
        self.window = window
        self.ex = cf.ThreadPoolExecutor(max_workers=workers)
        self.fut = {}
        self.next = 0
        self._fill()

    def _fill(self):
        while self.next < len(self.reqs) and len(self.fut) < self.window:
            rq = self.reqs[self.next]
            self.fut[rq.rid] = self.ex.submit(inputs.materialize, rq.problem)
            self.next += 1

    def get(self, rq):
        p = self.fut.pop(rq.rid).result()
        self._fill()
        return p

    def close(self):
        self.ex.shutdown(wait=False, cancel_futures=True)


TUNE_SIZES = (128, 181, 256, 362, 512, 724, 1024)


def tune_shapes(precision="fp32", steps=20, seed=11, sizes=TUNE_SIZES):
    """Tune the pool's batched 2D tile shapes (vklb_pool_autotune) on one
    two-state request per system and half-octave grid size of the request
    stream's 2D range; the library keeps the table for the process, so every
    pool created afterwards uses it. Returns the table."""
    samples = [inputs.random_riemann(system, 2, n, seed=seed * 100 + i * 10 + k, max_steps=steps)
               for i, system in enumerate(("sw", "euler", "mhd")) for k, n in enumerate(sizes)]
    pool = vklb.Pool(1 << 24, precision)
    try:
        return pool.autotune(samples, steps=steps)
    finally:
        pool.close()


def _alg_bytes(prob, precision):
    """Algorithmic bytes of one cell-step: every population read once and
    written once, 2 Q p s."""
    return 2 * prob.Q * prob.p * (4 if precision == "fp32" else 8)


def run_batched(requests, budget_bytes, precision="fp32", chunk_rounds=64, realtime=True, keep_results=False,
                progress=None):
    """Serve `requests` (inputs.Request, sorted by arrival) through a pool,
    `chunk_rounds` rounds per vklb_pool_run between polls (64 measured best
    on the seed-1 stream: 2 % more capacity than 32 and no worse latency at
    80 % load); progress(done, total) is called after every 200th completion."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    pool = vklb.Pool(budget_bytes, precision)
    pre = _Prefetch(reqs)
    pending = collections.deque(reqs)
    arrival = {}
    latencies = []
    results = {}
    cell_steps = 0
    alg_bytes = 0
    n_done = 0
    failed = []
    t0 = time.perf_counter()
    try:
        while n_done < len(reqs):
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                rq = pending.popleft()
                prob = pre.get(rq)
                arrival[rq.rid] = rq.arrival if realtime else 0.0
                pool.submit(prob, tag=rq.rid)
            st = pool.stats()
            if st["resident"] + st["queued"] == 0:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (time.perf_counter() - t0))))
                continue
            pool.run(chunk_rounds)
            for c in pool.poll():
                t_done = time.perf_counter() - t0
                latencies.append(t_done - arrival[c["tag"]])
                cell_steps += c["problem"].cells * c["steps"]
                alg_bytes += c["problem"].cells * c["steps"] * _alg_bytes(c["problem"], precision)
                n_done += 1
                if progress and n_done % 200 == 0:
                    progress(n_done, len(reqs))
                if c["status"] != 0:
                    failed.append((c["tag"], c["problem"].name, c["fail_step"], c["fail_cell"]))
                if keep_results:
                    results[c["tag"]] = (c["U"], c["t"], c["steps"], c["status"])
        makespan = time.perf_counter() - t0
        stats = pool.stats()
    finally:
        pre.close()
        pool.close()
    p50, p99 = _percentiles(latencies)
    ok = n_done - len(failed)
    return {"mode": "batched", "solves": n_done, "ok": ok, "makespan_s": makespan, "solves_per_s": ok / makespan,
            "completed_per_s": n_done / makespan,
            "p50_s": p50, "p99_s": p99, "cell_steps": cell_steps, "mcell_steps_per_s": cell_steps / makespan / 1e6,
            "alg_gb_per_s": alg_bytes / makespan / 1e9,
            "nonphysical": len(failed), "failed": failed, "arena_peak_bytes": stats["arena_peak"],
            "rounds": stats["rounds"], "graph_launches": stats["graph_launches"],
            "graph_captures": stats["graph_captures"],
            "results": results if keep_results else None}


def run_plain(requests, precision="fp32", realtime=True, keep_results=False, graph_chunk=0, progress=None):
    """One solve at a time in arrival order through the single-solve path
    (graph_chunk 0: its default graph chunks; -1: one plain launch per step);
    progress(done, total) is called after every 100th solve."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    pre = _Prefetch(reqs)
    latencies = []
    results = {}
    cell_steps = 0
    alg_bytes = 0
    failed = []
    t0 = time.perf_counter()
    try:
        for rq in reqs:
            prob = pre.get(rq)
            now = time.perf_counter() - t0
            if realtime and rq.arrival > now:
                time.sleep(rq.arrival - now)
            s = vklb.Solver(prob, precision=precision, graph_chunk=graph_chunk)
            s.init()
            try:
                U, t, n = s.run()
                status = 0
            except vklb.VklbError as e:
                # a non-physical state ends the solve, as it does in the pool
                if e.status != vklb.ERR_NONPHYSICAL:
                    raise
                d = s.diagnostics()
                U, t, n, status = None, d["t"], d["steps"], e.status
                failed.append((rq.rid, prob.name, d["fail_step"], d["fail_cell"]))
            s.close()
            t_done = time.perf_counter() - t0
            latencies.append(t_done - (rq.arrival if realtime else 0.0))
            cell_steps += prob.cells * n
            alg_bytes += prob.cells * n * _alg_bytes(prob, precision)
            if progress and len(latencies) % 100 == 0:
                progress(len(latencies), len(reqs))
            if keep_results:
                results[rq.rid] = (U, t, n, status)
        makespan = time.perf_counter() - t0
    finally:
        pre.close()
    p50, p99 = _percentiles(latencies)
    ok = len(reqs) - len(failed)
    return {"mode": "plain", "solves": len(reqs), "ok": ok, "makespan_s": makespan, "solves_per_s": ok / makespan,
            "completed_per_s": len(reqs) / makespan,
            "p50_s": p50, "p99_s": p99, "cell_steps": cell_steps, "mcell_steps_per_s": cell_steps / makespan / 1e6,
            "alg_gb_per_s": alg_bytes / makespan / 1e9,
            "nonphysical": len(failed), "failed": failed, "results": results if keep_results else None}


def with_arrivals(requests, rate, seed=7):
    """Re-time a request list as a Poisson process of the given rate (per s)."""
    rng = inputs.SplitMix64(seed)
    t = 0.0
    out = []
    for rq in requests:
        out.append(inputs.Request(rid=rq.rid, arrival=t, problem=rq.problem, steps=rq.steps))
        t += rng.exponential(rate)
    return out
