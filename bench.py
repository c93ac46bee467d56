#!/usr/bin/env python3
"""Benchmark of the nDGP scalar-field multigrid solve on one MI355X.

One step = one whole solve of the domain grid to ||S - L phi|| / ||S|| <= 1e-10
(source preparation, nested start, FAS V-cycles, norms, gauge) followed by the
fifth force, on the 512^3 periodic grid of the mixed-precision configuration
(box 512 Mpc/h, r_c H0 = 1, Omega_m = 0.3, lognormal delta with sigma_ln = 2.5
and P(k) ~ k^-2, seeded synthetic input resident in HBM), in FP64.
``--workload 256`` times the 256^3 grid with sigma_ln = 2 plus 50 top-hats
instead.

value = cell-updates/s = n^3 (nu1 + nu2) cycles / wall time per step.  The
timed steps run without the library's profiling flag.

The JSON line also carries:
  roofline      the red-black relaxation kernel of the finest level, timed
                with HIP events on its launch stream in a separate profiled
                pass after the timed steps; algorithmic bytes per cell update
                = 24 (read phi and S, write phi; FP64); beside the 8 TB/s
                peak, the measured copy ceiling: a plain stream that reads two
                n^3 FP64 arrays and writes one (24 B per cell), timed here;
  cpu_baseline  the CPU oracle's time to the same tolerance on the 32^3
                configuration and on the timed input;
  extra         patches: 256^3 + two nested 128^3 patches, full vs interpolated
                vs mixed + interpolated (time to tolerance, force difference);
                truncation: 256^3 + four nested 128^3 patches at the truncation
                levels l_d+1, l_d+2, l_d+4 and full, cell-wise truncation,
                G_eff per level; particles: one time step around the solver
                (cloud-in-cell density, nDGP and Newtonian solves, total force,
                cloud-in-cell force); amr: boxes placed on N_ref flags and
                solved as a tree (small boxes one workgroup each, in one
                launch per tree level) against box by box; large: 512^3
                solves at three r_c, FP64 and mixed; medium: the 256^3 solve;
                serving: the request stream (Poisson arrivals) and saturation,
                against the same requests solved one at a time.

    python bench.py [--steps K] [--warmup W] [--workload 512|256] [--no-extra] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nDGP MG cell-updates/s + HBM GB/s vs peak; served solves/s, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE_FP64 = 24.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ndgp_kernels.hip", "ndgp_internal.h", "ndgp_device.h"):
        with open(os.path.join(ROOT, "paper_1511_08200_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(n: int):
    """Measured HBM bytes per relaxation launch (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, calibrated by a copy kernel), if taken on the current kernels."""
    path = os.path.join(ROOT, "profiles", "smoother_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(str(n))


def workload(name, **kw):
    """A named workload of the package's presets (grid, parameters, seeded input)."""
    from paper_1511_08200_amd import presets
    return presets.load(name, **kw)


def solve_steps(ndgp, torch, grid, params, deltas, steps, warmup, with_force=True,
                median=False):
    """Time `steps` solves (+ force) after `warmup` untimed ones: the mean over
    the steps between two synchronisations, or (median=True, for the extras)
    the median of the steps each timed between synchronisations, which a
    stray pause of the host does not move."""
    dd = [torch.from_numpy(d).to("cuda") if d is not None else None for d in deltas]
    phi = ndgp.alloc_phi(grid)
    ws = ndgp.workspace(ndgp.workspace_bytes(grid, params))
    reps = []
    for _ in range(warmup):
        ndgp.solve(grid, params, dd, phi=phi, ws=ws)
        if with_force:
            ndgp.force(grid, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    each = []
    for _ in range(steps):
        t1 = time.perf_counter()
        _, rep = ndgp.solve(grid, params, dd, phi=phi, ws=ws)
        if with_force:
            ndgp.force(grid, phi)
        reps.append(rep)
        if median:
            torch.cuda.synchronize()
            each.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    if median and each:
        dt = float(np.median(each))
    return dt, reps, phi, dd


def kernel_name(cells, n):
    if cells == n**3:
        tz = 32 if n >= 256 else 4
        return (f"k_sweep_fused<64, 16, {tz}, 512, false> (one red-black sweep per launch, "
                "LDS-streamed, FP64; the variant with the coarse-grid correction on load is "
                "not in the timed set)")
    return "k_smooth_half (one colour per launch, FP64)"


def roofline(reps, n, copy_gbs=None):
    launches = sum(r.smooth_launches for r in reps)
    t_ms = sum(r.t_smooth_ms for r in reps)
    if not launches or t_ms <= 0:
        return None
    cells = reps[0].smooth_cells_per_launch
    avg_s = t_ms / 1e3 / launches
    alg_bytes = BYTES_PER_UPDATE_FP64 * cells
    achieved = alg_bytes / avg_s / 1e9
    tr = traffic_from_profiles(n)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": tr, "kernel": kernel_name(cells, n),
           "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
           "cells_per_launch": cells, "alg_bytes_per_launch": alg_bytes,
           "cell_updates_per_s": cells / avg_s}
    if copy_gbs:
        out["copy_ceiling_gbs"] = round(copy_gbs, 1)
        out["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return out


def copy_ceiling(torch, n, reps=5):
    """Measured stream ceiling for the relaxation's access pattern: read two
    n^3 FP64 arrays and write one (24 B per cell), as one elementwise kernel,
    timed with events on torch's stream (where it runs)."""
    a = torch.ones(n**3, dtype=torch.float64, device="cuda")
    b = torch.full_like(a, 2.0)
    c = torch.empty_like(a)
    for _ in range(2):
        torch.add(a, b, out=c)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        torch.add(a, b, out=c)
    ev[1].record()
    torch.cuda.synchronize()
    s = ev[0].elapsed_time(ev[1]) / 1e3 / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 24.0 * n**3 / s / 1e9


def cpu_baseline(cases):
    """The oracle (plain FP64 C, OpenMP) on the host: nested start + V(2,2)
    cycles to the same tolerance, on each (label, delta, h, rc) case."""
    from oracle import oracle as O
    rows = []
    for label, delta, h, rc in cases:
        beta = O.beta_lcdm(1.0, 0.3, rc)
        S, _ = O.source(delta, 0.3, 1.0, beta)
        n = delta.shape[0]
        log(f"cpu baseline: oracle on {label}")
        t0 = time.perf_counter()
        _, info = O.solve_periodic(S, h, O.alpha(rc, beta, 1.0), tol=1e-10)
        dt = time.perf_counter() - t0
        rows.append({"case": label, "s_to_tol": round(dt, 3), "cycles": info.cycles,
                     "rel_res": info.rel_res, "cell_updates_per_s": n**3 * 4 * info.cycles / dt})
    head = rows[-1]
    return {"value": head["cell_updates_per_s"], "unit": "cell-updates/s",
            "cores": O.num_threads(), "kind": "oracle",
            "sample": "; ".join(f"{r['case']}: nested start + {r['cycles']} V(2,2) cycles to "
                                f"rel. residual {r['rel_res']:.2e} in {r['s_to_tol']} s"
                                for r in rows),
            "time_to_tol_s": {r["case"]: r["s_to_tol"] for r in rows}}


def patch_workload(ndgp, torch, steps, depth):
    """256^3 domain + `depth` nested 128^3 patches (2x, 4x, ... resolution)
    centred on the largest top-hat.  depth 2: the full and the interpolated
    mode and mixed precision with interpolated patches, with the force
    difference.  depth 4: every truncation level (the paper's l_trunc = l_d + 1,
    2, 4 and the full run, Table I), cell-wise truncation, and G_eff per
    level; force differences of each truncated run against the full one."""
    rc = 1.0
    w = workload("nested-256" if depth == 2 else "nested-256-deep")
    assert len(w.grid.patches) == depth
    grid, deltas = w.grid, w.deltas()
    chain = [p.origin for p in grid.patches]
    if depth == 2:
        out = {"workload": "256^3 + 2 nested 128^3 patches (2x, 4x), lognormal sigma 2 + 50 "
                           "top-hats, r_cH0=1, tol 1e-10; FP64 full, FP64 interpolated, mixed "
                           "precision interpolated"}
        runs = (("full", ndgp.MODE_FULL, 0, ndgp.PREC_FP64),
                ("interpolated", ndgp.MODE_INTERPOLATED, 0, ndgp.PREC_FP64),
                ("mixed_interpolated", ndgp.MODE_INTERPOLATED, 0, ndgp.PREC_MIXED))
    else:
        out = {"workload": f"256^3 + {depth} nested 128^3 patches (2x..{2**depth}x), lognormal "
                           "sigma 2 + 50 top-hats, r_cH0=1, tol 1e-10; truncation levels 1 (all "
                           f"interpolated), 2, 4, {depth + 1} (full); mixed precision with every "
                           "patch interpolated; cell-wise truncation at F5/F_GR thresholds 0.02, "
                           "0.05, 0.08; G_eff per level"}
        runs = (("full", ndgp.MODE_FULL, 0, ndgp.PREC_FP64),
                ("trunc4", ndgp.MODE_TRUNCATED, 4, ndgp.PREC_FP64),
                ("trunc2", ndgp.MODE_TRUNCATED, 2, ndgp.PREC_FP64),
                ("interpolated", ndgp.MODE_INTERPOLATED, 0, ndgp.PREC_FP64),
                ("mixed_interpolated", ndgp.MODE_INTERPOLATED, 0, ndgp.PREC_MIXED))
    out["origins"] = [list(o) for o in chain]
    res = {}
    for name, mode, k, prec in runs:
        params = ndgp.Params(rc=rc, tol=1e-10, mode=mode, trunc_level=k, precision=prec)
        dt, reps, phi, dd = solve_steps(ndgp, torch, grid, params, deltas, steps, 1, median=True)
        res[name] = [p.clone() for p in phi]
        out[name] = {"ms_to_tol": round(dt * 1e3, 2), "cycles": reps[-1].cycles,
                     "rel_res": reps[-1].rel_res}
        del phi, dd
    t_full = out["full"]["ms_to_tol"]
    out["speedup_vs_full"] = {k: round(t_full / out[k]["ms_to_tol"], 2)
                              for k, _, _, _ in runs if k != "full"}
    out["speedup_interpolated_vs_full"] = out["speedup_vs_full"]["interpolated"]
    # mixed precision + interpolated levels against the plain FP64 full solve
    out["speedup_mixed_interpolated_vs_fp64_full"] = out["speedup_vs_full"]["mixed_interpolated"]
    a, b = res["mixed_interpolated"][0], res["interpolated"][0]
    out["mixed_vs_fp64_domain_rel_l2"] = float(torch.linalg.vector_norm(a - b)
                                               / torch.linalg.vector_norm(b))
    # force of each truncated run against the fully relaxed one (Eqs. errors,
    # errors2): relative to the full fifth force and to the GR force, whose
    # potential solves lap Psi = (3 beta / 2) S, i.e. 3 beta / 2 times the r_c = 0 field
    beta = ndgp.beta_lcdm(1.0, 0.3, rc)
    phi_gr, _ = ndgp.solve(grid, ndgp.Params(rc=0.0, beta=beta, tol=1e-10),
                           [torch.from_numpy(d).to("cuda") for d in deltas])
    # cell-wise truncation (Sec. III.C): iterate a patch cell only where its
    # parent's fifth force is at least a fraction of the Newtonian force
    # (Psi_N = 3 beta / 2 times the r_c = 0 field)
    psi = [1.5 * beta * p for p in phi_gr]
    dd = [torch.from_numpy(d).to("cuda") for d in deltas]
    full_params = ndgp.Params(rc=rc, tol=1e-10)
    ws = ndgp.workspace(ndgp.workspace_bytes(grid, full_params))
    thresholds = (0.02, 0.05, 0.08) if depth > 2 else ()
    if thresholds:
        out["cellwise"] = {}
    for thr in thresholds:
        phi_c = ndgp.alloc_phi(grid)
        ndgp.solve_cellwise(grid, full_params, dd, psi, thr, phi=phi_c, ws=ws)
        torch.cuda.synchronize()
        each = []
        for _ in range(steps):  # the median step, as for the modes above
            t0 = time.perf_counter()
            _, rep_c = ndgp.solve_cellwise(grid, full_params, dd, psi, thr, phi=phi_c, ws=ws)
            ndgp.force(grid, phi_c)
            torch.cuda.synchronize()
            each.append(time.perf_counter() - t0)
        dtc = float(np.median(each))
        name = f"cellwise{thr:g}"
        res[name] = phi_c
        out["cellwise"][f"{thr:g}"] = {"ms_to_tol": round(dtc * 1e3, 2), "cycles": rep_c.cycles,
                                       "iterated_fraction": rep_c.iterated_fraction,
                                       "speedup_vs_full": round(t_full / (dtc * 1e3), 2)}
    del ws, dd
    F_full = ndgp.force(grid, res["full"])
    F_lin = ndgp.force(grid, phi_gr)
    gr2 = []
    for lvl in range(1, depth + 1):
        _, g2, _ = ndgp.diff_norms(F_lin[lvl])
        gr2.append(g2 * (3 * beta) ** 2)
    # G_eff = 1 + |F5| / |F_GR| per level, each cell on the finest level that
    # holds it (the cell analogue of Fig. 3): mean and 16/50/84 percentiles
    # from a histogram with 100 log bins per decade
    edges = np.logspace(-4, 0, 201)

    def pct(h, q):
        c = np.cumsum(h) / h.sum()
        b = int(np.searchsorted(c, q))
        return float(edges[min(max(b - 1, 0), len(edges) - 1)])

    out["g_eff_per_level"] = {}
    for name in (("full", "trunc2", "interpolated", "cellwise0.08") if depth > 2
                 else ("full", "interpolated")):
        lv, hist = ndgp.geff_stats(grid, res[name], psi, edges)
        out["g_eff_per_level"][name] = [
            {"level": l, "cells": lv[l]["cells"], "mean_g_eff": 1.0 + lv[l]["mean"],
             "p16_84": [1.0 + pct(hist[l], 0.16), 1.0 + pct(hist[l], 0.84)],
             "median": 1.0 + pct(hist[l], 0.5)} for l in range(len(lv))]
    out["force_difference"] = {}
    for name in [k for k, _, _, _ in runs if k not in ("full", "mixed_interpolated")] + \
            [f"cellwise{t:g}" for t in thresholds]:
        F_t = ndgp.force(grid, res[name])
        rows = []
        for lvl in range(1, depth + 1):
            dd2, ff2, _ = ndgp.diff_norms(F_t[lvl], F_full[lvl])
            rows.append({"level": lvl, "rel_to_F5_full": float(np.sqrt(dd2 / ff2)),
                         "rel_to_F_GR": float(np.sqrt(dd2 / gr2[lvl - 1])),
                         "F5_over_FGR": float(np.sqrt(ff2 / gr2[lvl - 1]))})
        out["force_difference"][name] = rows
        del F_t
    return out


def particle_workload(ndgp, torch, steps):
    """One time step of the paper's loop around the solver (Sec. IV.A): 256^3
    equal-mass particles sampled from the 256^3 benchmark field, their
    cloud-in-cell density on the domain, the nDGP solve to 1e-10, the
    Newtonian potential (r_c = 0 solve), the total force and its
    cloud-in-cell interpolation back to the particles."""
    from paper_1511_08200_amd import synth
    w = workload("periodic-256")
    n, rc, f, grid = w.grid.n, 1.0, w.field, w.grid
    pos = torch.from_numpy(synth.make_particles(f, n**3, 7)).to("cuda")
    beta = ndgp.beta_lcdm(1.0, 0.3, rc)
    p5 = ndgp.Params(rc=rc, tol=1e-10)
    pn = ndgp.Params(rc=0.0, beta=beta, tol=1e-10)
    delta = ndgp.cic_density(grid, pos)
    phi, psi = ndgp.alloc_phi(grid), ndgp.alloc_phi(grid)
    ws = ndgp.workspace(ndgp.workspace_bytes(grid, p5))
    out = torch.empty_like(pos)
    stages = {"cic_density": 0.0, "solve_ndgp": 0.0, "solve_newton": 0.0, "total_force": 0.0,
              "cic_force": 0.0}
    reps = None
    for it in range(steps + 1):
        t = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ndgp.cic_density(grid, pos, delta=delta)
        torch.cuda.synchronize()
        t["cic_density"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, reps = ndgp.solve(grid, p5, delta, phi=phi, ws=ws)
        t["solve_ndgp"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, repn = ndgp.solve(grid, pn, delta, phi=psi, ws=ws)
        psi[0].mul_(1.5 * beta)  # Psi_N = (3 beta / 2) x the r_c = 0 field
        torch.cuda.synchronize()
        t["solve_newton"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        F = ndgp.total_force(grid, phi, psi)
        torch.cuda.synchronize()
        t["total_force"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        ndgp.cic_force(grid, F, pos, out=out)
        torch.cuda.synchronize()
        t["cic_force"] = time.perf_counter() - t0
        if it:  # the first pass warms up
            for k in stages:
                stages[k] += t[k] / steps
    total = sum(stages.values())
    # the same particles sorted by cell, as a tree code keeps them: the
    # deposit's atomics and the gather's reads then stay local
    pos_sorted = torch.from_numpy(synth.make_particles(f, n**3, 7, cell_order=True)).to("cuda")
    ndgp.cic_density(grid, pos_sorted, delta=delta)
    ndgp.cic_force(grid, F, pos_sorted, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ndgp.cic_density(grid, pos_sorted, delta=delta)
    torch.cuda.synchronize()
    dep_sorted = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        ndgp.cic_force(grid, F, pos_sorted, out=out)
    torch.cuda.synchronize()
    gat_sorted = (time.perf_counter() - t0) / steps
    return {"cell_ordered_particles_ms": {"cic_density": round(dep_sorted * 1e3, 3),
                                          "cic_force": round(gat_sorted * 1e3, 3)},
            "workload": "256^3 particles sampled from the 256^3 field (lognormal sigma 2 + 50 "
                        "top-hats, box 256 Mpc/h): CIC density, nDGP solve to 1e-10, Newtonian "
                        "solve, total force, CIC force at the particles",
            "ms": {k: round(v * 1e3, 3) for k, v in stages.items()},
            "ms_per_step": round(total * 1e3, 2),
            "particles_per_s_deposit": n**3 / stages["cic_density"],
            "particles_per_s_gather": n**3 / stages["cic_force"],
            "ndgp_cycles": reps.cycles[0], "newton_cycles": repn.cycles[0],
            "max_delta": float(delta[0].max())}


def amr_workload(ndgp, torch, steps):
    """Adaptive refinement (Sec. IV.A): a 256^3 field with small-scale
    clustering (lognormal sigma_ln 0.8 + 50 top-hats, box 256 Mpc/h), the
    cells holding more than N_ref = 16 of 256^3 particles flagged, cubic boxes
    placed on the flags (Berger-Rigoutsos, efficiency 0.7), every box relaxed
    to 1e-10 from its parent (full) or interpolated; the full solve also box
    by box (NDGP_TWO_PASS) against the small boxes in one launch."""
    from paper_1511_08200_amd import synth
    n, rc, n_ref = 256, 1.0, 16.0
    f = synth.make_field(n, 0.8, 1513, n_tophats=50)
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n))
    d0 = torch.from_numpy(f.delta).to("cuda")
    flags, counts = ndgp.refine_flags(grid, [d0], n**3, n_ref)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    boxes = ndgp.refine_boxes(flags[0], n, periodic=True, efficiency=0.7)
    t_cluster = time.perf_counter() - t0
    sizes = {}
    for b in boxes:
        sizes[str(b.n)] = sizes.get(str(b.n), 0) + 1
    dd = [d0] + [torch.from_numpy(synth.patch_delta(f, n, [b.origin], b.n)).to("cuda")
                 for b in boxes]
    out = {"workload": "256^3, lognormal sigma 0.8 + 50 top-hats, N_ref = 16 of 256^3 particles, "
                       "boxes by Berger-Rigoutsos (efficiency 0.7), r_cH0=1, tol 1e-10",
           "flagged_cells": int(counts[0]), "boxes": len(boxes), "box_sizes": sizes,
           "clustering_ms": round(t_cluster * 1e3, 1)}
    runs = (("full", ndgp.Params(rc=rc, tol=1e-10), steps),
            ("interpolated", ndgp.Params(rc=rc, tol=1e-10, mode=ndgp.MODE_INTERPOLATED), steps),
            ("full_box_by_box", ndgp.Params(rc=rc, tol=1e-10, two_pass=True), 1))
    res = {}
    for name, params, reps in runs:
        ws = ndgp.workspace(ndgp.amr_workspace_bytes(grid, params, boxes))
        phi, rep, per = ndgp.solve_amr(grid, params, boxes, dd, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            phi, rep, per = ndgp.solve_amr(grid, params, boxes, dd, phi=phi, ws=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        cyc = [p["cycles"] for p in per]
        out[name] = {"ms_to_tol": round(dt * 1e3, 2), "domain_cycles": rep.cycles[0],
                     "box_cycles_mean": round(float(np.mean(cyc)), 2), "box_cycles_max": max(cyc)}
        res[name] = phi
        del ws
    out["small_boxes_in_one_launch_speedup"] = round(out["full_box_by_box"]["ms_to_tol"] /
                                                     out["full"]["ms_to_tol"], 1)
    out["bitwise_equal_to_box_by_box"] = all(torch.equal(a, b) for a, b in
                                             zip(res["full"], res["full_box_by_box"]))
    return out


def large_workload(ndgp, torch, steps):
    """512^3 periodic, sigma_ln = 2.5, FP64, r_c H0 in {0.5, 1, 5}."""
    log("generating 512^3 input")
    w = workload("periodic-512")
    n, f, grid = w.grid.n, w.field, w.grid
    out = {"workload": "512^3 periodic, lognormal sigma 2.5, tol 1e-10, FP64 and mixed"}
    for rc in (0.5, 1.0, 5.0):
        params = ndgp.Params(rc=rc, tol=1e-10)
        dt, reps, phi, dd = solve_steps(ndgp, torch, grid, params, [f.delta], steps, 1,
                                        with_force=False)
        cyc = reps[-1].cycles[0]
        ent = {"fp64_ms_to_tol": round(dt * 1e3, 1), "fp64_cycles": cyc,
               "fp64_cell_updates_per_s": n**3 * 4 * cyc / dt}
        phi64 = phi[0].clone()
        del phi
        pm = ndgp.Params(rc=rc, tol=1e-10, precision=ndgp.PREC_MIXED)
        dtm, repm, phim, _ = solve_steps(ndgp, torch, grid, pm, [f.delta], steps, 1,
                                         with_force=False)
        dd2, aa2, _ = ndgp.diff_norms(phim[0], phi64)
        ent.update({"mixed_ms_to_tol": round(dtm * 1e3, 1), "mixed_outer_iters": repm[-1].cycles[0],
                    "mixed_rel_res": repm[-1].rel_res[0],
                    "mixed_vs_fp64_rel_l2": float(np.sqrt(dd2 / aa2)),
                    "mixed_speedup_vs_fp64": round(dt / dtm, 3)})
        out[f"rc{rc:g}"] = ent
        del phim, phi64, dd
        torch.cuda.empty_cache()
    return out


def medium_workload(ndgp, torch, steps):
    """The 256^3 configuration: lognormal sigma 2 + 50 top-hats, FP64 to 1e-10
    plus the force, with its own profiled relaxation roofline."""
    w = workload("periodic-256")
    n, rc, f, grid = w.grid.n, 1.0, w.field, w.grid
    dt, reps, phi, dd = solve_steps(ndgp, torch, grid, w.params, [f.delta], steps, 2)
    _, preps, _, _ = solve_steps(ndgp, torch, grid, ndgp.Params(rc=rc, tol=1e-10, profile=True),
                                 [f.delta], 2, 0)
    cyc = reps[-1].cycles[0]
    return {"workload": "256^3 periodic, lognormal sigma 2 + 50 top-hats, r_cH0=1, FP64, tol "
                        "1e-10, + force",
            "ms_to_tol": round(dt * 1e3, 2), "cycles": cyc,
            "cell_updates_per_s": n**3 * 4 * cyc / dt, "roofline": roofline(preps, n)}


def serving_workload(ndgp, torch, count, rate, sat_count):
    """Request stream: Poisson arrivals, n in {32, 64, 128, 256}^3, r_c H0 in
    {0.5, 1, 2, 5}, sigma_ln in [1, 2.5], mixed precision + one interpolated
    2x patch each, 64 GB device budget; then the same kind of requests all
    arriving at once (throughput at saturation)."""
    from paper_1511_08200_amd import serving
    sw = workload("serving")
    trace = serving.make_trace(count=count, rate=rate)  # the preset's stream at these sizes
    log(f"serving {count} requests at {rate}/s")
    res, summ = serving.serve(trace, budget_bytes=sw.budget_bytes, max_active=sw.max_active,
                              log=log)
    out = {"workload": f"{count} requests, Poisson {rate}/s, n in 32..256, r_cH0 in "
                       "{0.5,1,2,5}, mixed + interpolated patch, 64 GB budget",
           "poisson": summ}
    trace2 = serving.make_trace(count=sat_count, seed=1517, all_at_once=True)
    log(f"serving {sat_count} requests arriving at once")
    res2, summ2 = serving.serve(trace2, budget_bytes=sw.budget_bytes, max_active=sw.max_active,
                                realtime=False, log=log)
    out["saturation"] = summ2
    log(f"the same {sat_count} requests one at a time")
    seq = serving.serve_one_at_a_time(trace2)
    out["one_at_a_time"] = seq
    out["saturation_speedup_vs_one_at_a_time"] = round(summ2["solves_per_s"] / seq["solves_per_s"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("256", "512"), default="512",
                    help="timed workload: the 512^3 lognormal sigma 2.5 field (default) or "
                         "256^3 lognormal + top-hats")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the timed solve (mixed: FP32 multigrid on the correction "
                         "inside the FP64 defect-correction loop; no relaxation roofline)")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extra", default="patches,truncation,particles,amr,large,medium,serving",
                    help="comma-separated extra workloads to run after the timed one")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-saturation", type=int, default=400)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 128 MiB device-to-device copy three times "
                         "(the reference kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this solver runs on a single MI355X "
              "(multi-GPU domain decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_08200_amd import ndgp
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    ndgp.lib()

    rc = 1.0
    prec = ndgp.PREC_MIXED if args.precision == "mixed" else ndgp.PREC_FP64
    if args.workload == "512":
        w = workload("periodic-512", rc=rc, precision=prec)
        wl = ("ndgp-512^3-fp64-lognormal-sigma2.5, box 512 Mpc/h, r_cH0=1, tol 1e-10, "
              "V(2,2) 7 levels, + force")
    else:
        w = workload("periodic-256", rc=rc, precision=prec)
        wl = ("ndgp-256^3-fp64-lognormal-sigma2+50tophats, box 256 Mpc/h, r_cH0=1, tol 1e-10, "
              "V(2,2) 6 levels, + force")
    n, grid, params = w.grid.n, w.grid, w.params
    log(f"generating {n}^3 input")
    f = w.field
    if prec == ndgp.PREC_MIXED:
        wl = wl.replace("-fp64-", "-mixed-")
    log("timing")
    dt, reps, phi, dd = solve_steps(ndgp, torch, grid, params, [f.delta], args.steps,
                                    args.warmup)
    cycles = reps[-1].cycles[0]
    assert all(r.cycles[0] == cycles for r in reps)
    value = n**3 * 4 * cycles / dt
    del phi, dd
    # the roofline from a separate pass with the relaxation launches timed
    log("profiled pass (relaxation roofline)")
    _, preps, phi, dd = solve_steps(ndgp, torch, grid,
                                    ndgp.Params(rc=rc, tol=1e-10, profile=True, precision=prec),
                                    [f.delta], 3, 0)
    del phi, dd
    torch.cuda.empty_cache()
    log("copy ceiling")
    copy_gbs = copy_ceiling(torch, n)
    line = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == ndgp.PREC_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": wl, "n": n, "cycles": cycles, "rel_res": reps[-1].rel_res[0],
                   "solves_per_s": 1.0 / dt},
        "roofline": roofline(preps, n, copy_gbs),
    }
    if args.calibrate_copy:
        a = torch.ones(n**3, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = {"read": a.numel() * 8, "write": b.numel() * 8}
        del a, b
    if not args.no_cpu:
        w32 = workload("periodic-32")
        line["cpu_baseline"] = cpu_baseline(
            [("32^3 sigma 1 (box 64 Mpc/h)", w32.field.delta, w32.grid.h, 1.0),
             (f"{n}^3 timed input", f.delta, grid.h, rc)])
    extras = set() if args.no_extra else {e for e in args.extra.split(",") if e}
    unknown = extras - {"patches", "truncation", "particles", "amr", "large", "medium", "serving"}
    if unknown:
        raise SystemExit(f"unknown extra workloads: {sorted(unknown)}")
    if extras:
        out = line.setdefault("extra", {})
        if "patches" in extras:
            log("patch workload")
            out["patches"] = patch_workload(ndgp, torch, 5, 2)
        if "truncation" in extras:
            log("truncation workload")
            out["truncation"] = patch_workload(ndgp, torch, 5, 4)
        if "particles" in extras:
            log("particle workload")
            out["particles"] = particle_workload(ndgp, torch, 3)
        if "amr" in extras:
            log("adaptive refinement workload")
            out["amr"] = amr_workload(ndgp, torch, 3)
        if "large" in extras:
            log("512^3 workload")
            out["large"] = large_workload(ndgp, torch, 3)
        if "medium" in extras:
            log("256^3 workload")
            out["medium"] = medium_workload(ndgp, torch, 5)
        if "serving" in extras and args.serve_requests > 0:
            out["serving"] = serving_workload(ndgp, torch, args.serve_requests,
                                              args.serve_rate, args.serve_saturation)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
