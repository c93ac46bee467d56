"""Continuous-batching request loop over the library's non-blocking plans.

Requests arrive over time (Poisson arrivals), each asking for one nDGP solve of
its own grid size, r_c and density.  The loop admits a waiting request as soon
as a stream slot is free and its device memory fits the HBM budget, keeps every
admitted solve in flight on its own HIP stream, and round-robins them: poll a
plan (never blocks), give it its next V-cycle when it is waiting, retire it
when it is done and admit the next request into the freed slot and memory.
Work of different solves overlaps on the device; each solve's result is bit
for bit what it would be alone, because a plan's cycle count depends only on
its own residual history and every kernel is deterministic.

Each request: lognormal density drawn on the device (seeded), one 2x patch of
(n/2)^3 cells centred on the densest cell, filled by interpolation (the
truncated mode of Sec. III.B), mixed precision by default.
"""
from __future__ import annotations

import dataclasses
import json
import time
from collections import deque

import numpy as np
import torch

from . import ndgp, synth


@dataclasses.dataclass
class Request:
    idx: int
    arrival: float   # seconds after the start of the run
    n: int
    rc: float
    sigma: float
    seed: int


@dataclasses.dataclass
class Result:
    idx: int
    n: int
    arrival: float
    admitted: float
    done: float
    cycles: int
    rel_res: float
    status: int
    bytes: int
    rc: float = 0.0
    sigma: float = 0.0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_trace(count: int = 2000, rate: float = 50.0, seed: int = 1516,
               sizes=(32, 64, 128, 256), rcs=(0.5, 1.0, 2.0, 5.0), sigma=(1.0, 2.5),
               all_at_once: bool = False) -> list:
    """Seeded request stream: exponential gaps of mean 1/rate (or every
    arrival at t = 0), size and r_c uniform over the given sets, sigma_ln
    uniform in the given range, request i drawing its density with seed
    100000 + i."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=count)
    rc = rng.choice(np.asarray(rcs), size=count)
    sg = rng.uniform(sigma[0], sigma[1], size=count)
    return [Request(i, 0.0 if all_at_once else float(t[i]), int(ns[i]), float(rc[i]),
                    float(sg[i]), 100000 + i) for i in range(count)]


def request_grid(req: Request, flat: int, precision=ndgp.PREC_MIXED, tol: float = 1e-10,
                 box_per_cell: float = 1.0):
    """Grid and parameters of one request whose densest cell has the flat
    index `flat`: one (n/2)^3 patch at twice the resolution centred there."""
    n = req.n
    k, j, i = flat // (n * n), (flat // n) % n, flat % n
    cover = n // 4  # the (n/2)^3 patch at twice the resolution covers (n/4)^3 cells
    origin = (i - cover // 2, j - cover // 2, k - cover // 2)
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(box_per_cell * n, n),
                     patches=[ndgp.Patch(n // 2, origin)])
    params = ndgp.Params(rc=req.rc, tol=tol, mode=ndgp.MODE_INTERPOLATED, precision=precision)
    return grid, params


def request_problem(req: Request, device, precision=ndgp.PREC_MIXED, tol: float = 1e-10,
                    box_per_cell: float = 1.0):
    """Density, grid and parameters of one request (density made on the
    current stream of `device`; waits for its densest cell)."""
    delta = synth.lognormal_delta_torch(req.n, req.sigma, req.seed, device=device)
    grid, params = request_grid(req, int(torch.argmax(delta).item()), precision, tol,
                                box_per_cell)
    return delta, grid, params


def _shape_only(req: Request, precision, tol):
    """Grid and parameters of a request without its density (for sizing)."""
    n = req.n
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n), patches=[ndgp.Patch(n // 2, (0, 0, 0))])
    params = ndgp.Params(rc=req.rc, tol=tol, mode=ndgp.MODE_INTERPOLATED, precision=precision)
    return grid, params


def request_bytes(grid: ndgp.Grid, params: ndgp.Params) -> int:
    """Device bytes a request holds while it runs: workspace, density and
    solution arrays, plus the density generator's transient buffers."""
    n = grid.n
    cells = n ** 3 * 8
    patch = sum((p.n + 2) ** 3 * 8 for p in grid.patches)
    return ndgp.workspace_bytes(grid, params) + 2 * cells + patch + 3 * cells


class _Active:
    __slots__ = ("req", "plan", "stream", "admitted", "bytes", "delta", "grid", "params",
                 "where", "placed")


def warm_up(trace: list, precision=ndgp.PREC_MIXED, tol: float = 1e-10, device="cuda"):
    """One solve per grid size present in the trace (first-use set-up of the
    density generator's FFTs and of the kernels), outside any timing."""
    for n in sorted({r.n for r in trace}):
        req = Request(-1, 0.0, n, 1.0, 1.5, 99)
        delta, grid, params = request_problem(req, device, precision, tol)
        plan = ndgp.Plan(grid, params, [delta])
        while not plan.poll():
            plan.step()
        plan.close()
    torch.cuda.synchronize(device)


def serve(trace: list, budget_bytes: float = 64e9, max_active: int = 16,
          precision=ndgp.PREC_MIXED, tol: float = 1e-10, device="cuda",
          keep_results: bool = False, realtime: bool = True, log=None, warm: bool = True,
          request_log: str = None):
    """Run the request stream; returns (results, summary[, kept]) where kept
    maps request index -> (delta, phi list) when keep_results is set.
    ``request_log``: a path; one JSON line per finished request is appended
    (index, size, r_c, sigma, arrival / admission / completion times in
    seconds from the start, latency, cycles, residual, status, bytes held)."""
    if warm:
        warm_up(trace, precision, tol, device)
    log_fh = open(request_log, "a") if request_log else None
    streams = [torch.cuda.Stream(device=device) for _ in range(max_active)]
    free_streams = deque(range(max_active))
    pending = deque(sorted(trace, key=lambda r: (r.arrival, r.idx)))
    active: list = []
    results: list = []
    kept = {}
    used = 0
    peak_used = 0
    peak_active = 0
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    last_log = 0.0
    while pending or active:
        # admission: arrived requests, in order, while a slot and the budget allow
        while pending and free_streams and (not realtime or pending[0].arrival <= now()):
            req = pending[0]
            need = request_bytes(*_shape_only(req, precision, tol))
            if used + need > budget_bytes and active:
                break
            pending.popleft()
            si = free_streams.popleft()
            with torch.cuda.stream(streams[si]):
                # the density and its densest cell, copied back without waiting:
                # the plan is created once the copy has landed
                a = _Active()
                a.req, a.stream, a.admitted, a.bytes = req, si, now(), need
                a.delta = synth.lognormal_delta_torch(req.n, req.sigma, req.seed, device=device)
                a.where = torch.empty(1, dtype=torch.int64, pin_memory=True)
                a.where.copy_(torch.argmax(a.delta).reshape(1), non_blocking=True)
                a.placed = torch.cuda.Event()
                a.placed.record(streams[si])
                a.plan = None
            used += need
            peak_used = max(peak_used, used)
            active.append(a)
            peak_active = max(peak_active, len(active))
        # progress: poll every plan, step the waiting ones, retire the finished
        still = []
        for a in active:
            if a.plan is None:  # waiting for its densest cell
                if a.placed.query():
                    a.grid, a.params = request_grid(a.req, int(a.where[0]), precision, tol)
                    with torch.cuda.stream(streams[a.stream]):
                        a.plan = ndgp.Plan(a.grid, a.params, [a.delta], stream=streams[a.stream])
                still.append(a)
                continue
            if a.plan.poll():
                rep = a.plan.report
                results.append(Result(a.req.idx, a.req.n, a.req.arrival, a.admitted, now(),
                                      rep.cycles[0], rep.rel_res[0], rep.status, a.bytes,
                                      a.req.rc, a.req.sigma))
                if log_fh:
                    r = results[-1]
                    log_fh.write(json.dumps({
                        "idx": r.idx, "n": r.n, "rc": r.rc, "sigma": r.sigma,
                        "arrival_s": r.arrival, "admitted_s": r.admitted, "done_s": r.done,
                        "latency_ms": r.latency * 1e3, "cycles": r.cycles, "rel_res": r.rel_res,
                        "status": r.status, "bytes": r.bytes}) + "\n")
                if keep_results:
                    kept[a.req.idx] = (a.delta, a.plan.phi, a.grid, a.params)
                a.plan.close()
                used -= a.bytes
                free_streams.append(a.stream)
            else:
                a.plan.step()
                still.append(a)
        active = still
        if log and now() - last_log > 5.0:
            last_log = now()
            log(f"t={last_log:.1f}s done={len(results)} active={len(active)} "
                f"pending={len(pending)} used={used / 1e9:.2f} GB")
        if not active and pending and realtime:
            wait = pending[0].arrival - now()
            if wait > 0:
                time.sleep(min(wait, 0.002))
    torch.cuda.synchronize(device)
    if log_fh:
        log_fh.close()
    summary = summarize(results)
    summary.update({"peak_active": peak_active, "peak_bytes": peak_used,
                    "budget_bytes": budget_bytes, "max_active": max_active})
    if keep_results:
        return results, summary, kept
    return results, summary


def serve_one_at_a_time(trace: list, precision=ndgp.PREC_MIXED, tol: float = 1e-10,
                        device="cuda", warm: bool = True) -> dict:
    """The same requests solved one after the other with the blocking solve
    (density, densest cell, solve, next request): the baseline that the
    continuous-batching loop is measured against."""
    if warm:
        warm_up(trace, precision, tol, device)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    failed = 0
    for req in sorted(trace, key=lambda r: (r.arrival, r.idx)):
        delta, grid, params = request_problem(req, device, precision, tol)
        _, rep = ndgp.solve(grid, params, [delta], check=False)
        failed += rep.status != ndgp.NDGP_OK
    torch.cuda.synchronize(device)
    dt = time.perf_counter() - t0
    return {"completed": len(trace), "failed": int(failed), "solves_per_s": len(trace) / dt,
            "makespan_s": dt}


def summarize(results: list) -> dict:
    if not results:
        return {"completed": 0}
    lat = np.array([r.latency for r in results])
    first = min(r.arrival for r in results)
    last = max(r.done for r in results)
    by_n = {}
    for n in sorted({r.n for r in results}):
        ln = np.array([r.latency for r in results if r.n == n])
        by_n[str(n)] = {"count": int(len(ln)), "p50_ms": float(np.percentile(ln, 50) * 1e3),
                        "p99_ms": float(np.percentile(ln, 99) * 1e3)}
    failures = [{"idx": r.idx, "n": r.n, "rc": r.rc, "sigma": round(r.sigma, 3),
                 "status": r.status, "cycles": r.cycles, "rel_res": r.rel_res}
                for r in results if r.status != ndgp.NDGP_OK]
    return {"completed": len(results),
            "failed": len(failures),
            "failures": failures[:20],
            "solves_per_s": len(results) / max(last - first, 1e-9),
            "makespan_s": last - first,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_cycles": float(np.mean([r.cycles for r in results])),
            "by_n": by_n}
