"""The non-blocking plan API and the continuous-batching loop on the GPU."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1511_08200_amd import ndgp, serving, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-serving] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ndgp.lib()


@pytest.mark.parametrize("precision", [ndgp.PREC_FP64, ndgp.PREC_MIXED])
def test_plan_equals_blocking_solve(precision):
    """A plan driven by poll/step gives the same bits as ndgp_solve."""
    say(f"plan vs solve precision={precision}")
    n = 64
    f = synth.make_field(n, 2.0, 77, n_tophats=5)
    d = torch.from_numpy(f.delta).cuda()
    c = synth.densest_tophat_centre(f)
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(64.0, n),
                     patches=[ndgp.Patch(32, synth.patch_origin_centred(c, 16))])
    params = ndgp.Params(rc=2.0, tol=1e-10, mode=ndgp.MODE_INTERPOLATED, precision=precision)
    phi_a, rep_a = ndgp.solve(grid, params, [d])
    plan = ndgp.Plan(grid, params, [d])
    steps = 0
    while not plan.poll():
        plan.step()
        steps += 1
        assert steps < 10**6
    torch.cuda.synchronize()
    rep_b = plan.report
    assert rep_b.status == 0 and rep_b.cycles[0] == rep_a.cycles[0]
    assert rep_b.history == rep_a.history
    for x, y in zip(phi_a, plan.phi):
        assert torch.equal(x, y)
    plan.close()


def test_plan_destroyed_in_flight_leaves_later_plans_exact():
    """Plans destroyed with work still enqueued (after create, after a step)
    wait for it before their pinned norm slot is reused: the plans created
    next, which take those slots, still give the blocking solve's bits."""
    say("plan destroyed in flight")
    n = 64
    f = synth.make_field(n, 1.5, 78, n_tophats=3)
    d = torch.from_numpy(f.delta).cuda()
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(64.0, n))
    params = ndgp.Params(rc=1.0, tol=1e-10)
    phi_a, rep_a = ndgp.solve(grid, params, [d])
    side = torch.cuda.Stream()
    for stepped in (False, True):
        with torch.cuda.stream(side):
            doomed = [ndgp.Plan(grid, params, [d], stream=side) for _ in range(3)]
        for p in doomed:
            if stepped:
                side.synchronize()
                assert not p.poll()   # the first norm is in: the plan waits for a step
                p.step()              # one V-cycle and its norm enqueued
            p.close()                 # with that work still in flight
        plan = ndgp.Plan(grid, params, [d])
        while not plan.poll():
            plan.step()
        torch.cuda.synchronize()
        rep_b = plan.report
        assert rep_b.status == 0 and rep_b.history == rep_a.history
        assert torch.equal(plan.phi[0], phi_a[0])
        plan.close()


def _plan_to_end(grid, params, delta):
    plan = ndgp.Plan(grid, params, delta)
    steps = 0
    while not plan.poll():
        plan.step()
        steps += 1
        assert steps < 10**7
    torch.cuda.synchronize()
    return plan


@pytest.mark.parametrize("precision", [ndgp.PREC_FP64, ndgp.PREC_MIXED])
def test_plan_damped_and_safeguard_equal_blocking_solve(precision):
    """Plans follow the blocking solve bit for bit (a) with the damped step
    (NDGP_DAMPED) on the extreme request of the serving trace (sigma_ln 2.47,
    r_cH0 = 5, 1 Mpc/h cells), and (b) on a source with unphysical voids
    (delta = -40 in three cells: no elliptic solution near them, cells without
    a real root), which stagnates and ends with NDGP_ENOCONV: same status,
    cycles, restart cycle (if any), history and field."""
    say(f"plan damped precision={precision}")
    n, rc, sigma, seed = 256, 5.0, 2.4694042826895837, 100881
    d = synth.lognormal_delta_torch(n, sigma, seed, device="cuda")
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n))
    params = ndgp.Params(rc=rc, tol=1e-10, precision=precision, max_cycles=60, damped=True)
    phi_a, rep_a = ndgp.solve(grid, params, [d])
    plan = _plan_to_end(grid, params, [d])
    rep_b = plan.report
    say(f"  damped: cycles={rep_b.cycles[0]} damped_from={rep_b.damped_from[0]}")
    assert rep_b.status == 0 and rep_a.damped_from[0] == 1 == rep_b.damped_from[0]
    assert rep_b.cycles == rep_a.cycles and rep_b.history == rep_a.history
    assert torch.equal(phi_a[0], plan.phi[0])
    plan.close()
    # (b) the safeguard restart
    m = 32
    v = synth.make_field(m, 2.0, 61, n_tophats=4).delta.copy()
    for (i, j, k) in ((5, 6, 7), (20, 21, 3), (11, 27, 30)):
        v[k, j, i] = -40.0
    dv = torch.from_numpy(v).to("cuda")
    gv = ndgp.Grid(n=m, h=ndgp.cell_size(float(m), m))
    pv = ndgp.Params(rc=rc, tol=1e-10, precision=precision, max_cycles=40)
    phi_a, rep_a = ndgp.solve(gv, pv, [dv], check=False)
    plan = _plan_to_end(gv, pv, [dv])
    rep_b = plan.report
    say(f"  void: status={rep_a.status} cycles={rep_a.cycles[0]} "
        f"damped_from={rep_a.damped_from[0]} fallbacks={rep_a.fallbacks}")
    assert rep_a.status == ndgp.NDGP_ENOCONV == rep_b.status
    assert rep_a.fallbacks > 0 and rep_b.fallbacks == rep_a.fallbacks
    assert rep_b.damped_from == rep_a.damped_from and rep_b.cycles == rep_a.cycles
    assert np.array_equal(np.array(rep_b.history), np.array(rep_a.history), equal_nan=True)
    assert np.array_equal(plan.phi[0].cpu().numpy(), phi_a[0].cpu().numpy(), equal_nan=True)
    plan.close()


def test_plan_reports_bad_input():
    n = 32
    bad = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    bad[1, 2, 3] = float("inf")
    plan = ndgp.Plan(ndgp.Grid(n=n, h=1e-3), ndgp.Params(rc=1.0), [bad])
    with pytest.raises(ndgp.NdgpError) as e:
        while not plan.poll():
            plan.step()
    assert e.value.status == ndgp.NDGP_EINVAL
    plan.close()
    with pytest.raises(ndgp.NdgpError):  # full-mode patches are not served
        ndgp.Plan(ndgp.Grid(n=n, h=1e-3, patches=[ndgp.Patch(16, (8, 8, 8))]),
                  ndgp.Params(rc=1.0, mode=ndgp.MODE_FULL), [bad, bad[:16, :16, :16].contiguous()])


def test_continuous_batching_isolation():
    """Requests of mixed sizes and r_c run concurrently on several streams;
    each result equals the same request solved alone, bit for bit."""
    trace = serving.make_trace(count=24, rate=400.0, seed=9, sizes=(32, 64, 128))
    say("serving 24 requests, 6 slots")
    results, summary, kept = serving.serve(trace, budget_bytes=4e9, max_active=6,
                                           keep_results=True)
    say(f"summary {summary}")
    assert summary["completed"] == 24 and summary["failed"] == 0
    assert summary["peak_active"] >= 2
    for r in results:
        delta, phi_mix, grid, params = kept[r.idx]
        phi_alone, rep = ndgp.solve(grid, params, [delta])
        assert rep.cycles[0] == r.cycles
        for x, y in zip(phi_alone, phi_mix):
            assert torch.equal(x, y), f"request {r.idx} differs"


def test_budget_limits_admission():
    trace = serving.make_trace(count=6, rate=1e6, seed=3, sizes=(64,))
    one = serving.request_bytes(*serving._shape_only(trace[0], ndgp.PREC_MIXED, 1e-10))
    results, summary = serving.serve(trace, budget_bytes=1.5 * one, max_active=4)
    assert summary["completed"] == 6 and summary["peak_active"] == 1


def test_one_at_a_time_baseline():
    trace = serving.make_trace(count=6, seed=5, sizes=(32, 64), all_at_once=True)
    out = serving.serve_one_at_a_time(trace)
    assert out["completed"] == 6 and out["failed"] == 0 and out["solves_per_s"] > 0


def test_request_log(tmp_path):
    """One JSON line per finished request, with its timings and outcome."""
    import json
    trace = serving.make_trace(count=5, rate=1e6, seed=4, sizes=(32,))
    path = tmp_path / "requests.jsonl"
    results, summary = serving.serve(trace, budget_bytes=4e9, max_active=2,
                                     request_log=str(path))
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert summary["completed"] == 5 and len(lines) == 5
    assert sorted(x["idx"] for x in lines) == [r.idx for r in trace]
    for x in lines:
        assert x["status"] == 0 and x["cycles"] > 0
        assert x["arrival_s"] <= x["admitted_s"] <= x["done_s"]
        assert abs(x["latency_ms"] - 1e3 * (x["done_s"] - x["arrival_s"])) < 1e-6
