"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: FP64 solutions agree to a relative L2 error <= 1e-11 when both sides are
run to rounding-level stagnation (the tolerance the FP64 path is built for);
residuals, interpolation and forces agree element by element to rounding.
At the full 256^3 / 512^3 sizes, where the oracle cannot afford a solve, the
oracle evaluates the residual of the GPU answer (everywhere, and at sampled
cells against the GPU's own residual).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1511_08200_amd import ndgp, synth  # noqa: E402

pytestmark = pytest.mark.gpu

PHI_TOL = 1e-11


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ndgp.lib()  # fails loudly if the HIP library is missing


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def oracle_periodic(delta, h, rc, omega_m=0.3, a=1.0):
    beta = O.beta_lcdm(a, omega_m, rc)
    S, _ = O.source(delta, omega_m, a, beta)
    phi, info = O.solve_periodic(S, h, O.alpha(rc, beta, a))
    assert info.status == 0, info
    return phi, S


def gpu_solve(delta_list, grid, **kw):
    params = ndgp.Params(**kw)
    phi, rep = ndgp.solve(grid, params, [dev(d) if d is not None else None for d in delta_list])
    torch.cuda.synchronize()
    return [p.cpu().numpy() for p in phi], rep


# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,box,sigma,tophats,rc,seed", [
    (32, 64.0, 1.0, 0, 1.0, 1512),     # the 32^3 plain FP64 configuration
    (32, 64.0, 2.0, 4, 5.0, 7),
    (64, 64.0, 2.0, 20, 1.0, 8),       # lognormal + top-hats, several tiles
    (64, 128.0, 2.5, 0, 5.0, 9),       # strongest screening of the 512^3 set
    (16, 16.0, 1.0, 1, 0.5, 3),
    (8, 16.0, 1.0, 0, 1.0, 4),          # the smallest grid: one level, the coarsest solve only
    (128, 128.0, 2.0, 30, 1.0, 10),    # large enough for the fused LDS sweep
    (64, 64.0, 2.0, 10, 0.0, 11),      # r_c = 0: the linear Poisson equation
])
def test_periodic_solution_matches_oracle(n, box, sigma, tophats, rc, seed):
    say(f"periodic n={n} sigma={sigma} tophats={tophats} rc={rc}")
    f = synth.make_field(n, sigma, seed, n_tophats=tophats)
    h = ndgp.cell_size(box, n)
    phio, S = oracle_periodic(f.delta, h, rc)
    (phig,), rep = gpu_solve([f.delta], ndgp.Grid(n=n, h=h), rc=rc, tol=0.0, max_cycles=200)
    say(f"  cycles={rep.cycles[0]} rel_res={rep.rel_res[0]:.2e} fallbacks={rep.fallbacks}")
    assert rep.status == 0
    assert abs(phig.mean()) < 1e-15 * np.abs(phig).max()
    assert rel(phig, phio) <= PHI_TOL


def test_tolerance_stop_and_history():
    n = 32
    f = synth.make_field(n, 1.0, 1512)
    h = ndgp.cell_size(64.0, n)
    (phig,), rep = gpu_solve([f.delta], ndgp.Grid(n=n, h=h), rc=1.0, tol=1e-10)
    say(f"tol stop: cycles={rep.cycles[0]} hist={rep.history}")
    assert rep.status == 0 and rep.rel_res[0] <= 1e-10
    assert rep.cycles[0] <= 25
    assert len(rep.history) == rep.cycles[0]
    assert all(b < a for a, b in zip(rep.history, rep.history[1:]))
    # the oracle's residual of the GPU answer says the same
    beta = O.beta_lcdm(1.0, 0.3, 1.0)
    S, _ = O.source(f.delta, 0.3, 1.0, beta)
    r = S - O.operator(phig, h, O.alpha(1.0, beta, 1.0))
    assert np.linalg.norm(r) / np.linalg.norm(S) == pytest.approx(rep.rel_res[0], rel=1e-3)


@pytest.mark.parametrize("n,level_shape", [(32, None), (64, None)])
def test_residual_elementwise(n, level_shape):
    say(f"residual n={n}")
    rng = np.random.default_rng(n)
    f = synth.make_field(n, 2.0, 21, n_tophats=3)
    h = ndgp.cell_size(n * 1.0, n)
    rc = 2.0
    beta = O.beta_lcdm(1.0, 0.3, rc)
    S, _ = O.source(f.delta, 0.3, 1.0, beta)
    phi = rng.standard_normal((n, n, n)) * 1e-6
    ro = S - O.operator(phi, h, O.alpha(rc, beta, 1.0))
    grid = ndgp.Grid(n=n, h=h)
    r, relg = ndgp.residual(grid, ndgp.Params(rc=rc), [dev(f.delta)], dev(phi))
    rg = r.cpu().numpy()
    scale = np.abs(ro).max()
    assert np.abs(rg - ro).max() <= 1e-12 * scale
    assert relg == pytest.approx(np.linalg.norm(ro) / np.linalg.norm(S), rel=1e-12)


def test_zero_source_and_one_dimensional_source():
    n = 32
    h = ndgp.cell_size(64.0, n)
    say("zero source")
    (phig,), rep = gpu_solve([np.zeros((n, n, n))], ndgp.Grid(n=n, h=h), rc=1.0)
    assert rep.cycles[0] == 0 and np.all(phig == 0.0)
    say("1D source")
    rng = np.random.default_rng(12)
    rho = np.exp(2.0 * rng.standard_normal(n))
    prof = rho / rho.mean() - 1.0
    delta = np.broadcast_to(prof.reshape(1, 1, n), (n, n, n)).copy()
    (phig,), rep = gpu_solve([delta], ndgp.Grid(n=n, h=h), rc=5.0, tol=0.0, max_cycles=200)
    beta = O.beta_lcdm(1.0, 0.3, 5.0)
    S, _ = O.source(delta, 0.3, 1.0, beta)
    # discrete Poisson answer by FFT (the nonlinear term vanishes on 1D fields)
    m = np.fft.fftfreq(n) * n
    lam = -(4.0 / h**2) * np.sin(np.pi * m / n) ** 2
    lam[0] = 1.0
    pk = np.fft.fft(S[0, 0, :]) / lam
    pk[0] = 0.0
    ref = np.real(np.fft.ifft(pk))
    assert rel(phig[0, 0, :], ref) <= PHI_TOL
    assert np.abs(phig - phig[:1, :1, :]).max() <= 1e-13 * np.abs(ref).max()


def test_scale_law_bitwise_and_determinism():
    """h -> 2h with the same density gives exactly 4 phi (the kernels work in
    cell units and every step is homogeneous); a rerun gives the same bits."""
    n = 32
    f = synth.make_field(n, 2.0, 5, n_tophats=2)
    h = ndgp.cell_size(64.0, n)
    say("scale law")
    (p1,), r1 = gpu_solve([f.delta], ndgp.Grid(n=n, h=h), rc=1.0, tol=1e-12, max_cycles=100)
    (p2,), r2 = gpu_solve([f.delta], ndgp.Grid(n=n, h=2 * h), rc=1.0, tol=1e-12, max_cycles=100)
    (p3,), r3 = gpu_solve([f.delta], ndgp.Grid(n=n, h=h), rc=1.0, tol=1e-12, max_cycles=100)
    assert r1.cycles == r2.cycles
    assert np.array_equal(p2, 4 * p1)
    assert np.array_equal(p3, p1)


@pytest.mark.parametrize("n,levels", [(16, 0), (32, 0), (64, 0), (64, 5), (64, 6), (128, 0),
                                      (256, 0)])
def test_fused_kernels_bitwise_equal_per_level_launches(n, levels):
    """The one-launch LDS sweep (n >= 128) and the one-workgroup bottom of the
    V-cycle (levels of at most 16^3, coarsest 8^3, 4^3 or 2^3) give the same
    bits for the whole solve as one launch per colour, per transfer and per
    level."""
    say(f"fused vs per-level launches n={n} levels={levels}")
    f = synth.make_field(n, 2.0, 31, n_tophats=10)
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n))
    d = dev(f.delta)
    a, ra = ndgp.solve(grid, ndgp.Params(rc=1.0, tol=1e-10, n_levels=levels), [d])
    b, rb = ndgp.solve(grid, ndgp.Params(rc=1.0, tol=1e-10, n_levels=levels, two_pass=True),
                       [d])
    torch.cuda.synchronize()
    assert ra.cycles == rb.cycles and ra.history == rb.history
    assert ra.fallbacks == rb.fallbacks
    assert not any(ra.damped_from)  # the safeguard stays off for ordinary fields
    assert torch.equal(a[0], b[0])


@pytest.mark.parametrize("m,pn2,wrap", [(128, 128, False), (128, 64, True), (256, 128, False)])
def test_patch_fused_sweep_bitwise_equal_per_colour_launches(m, pn2, wrap):
    """The finest level of a refinement (fixed ghost shell) relaxed by the
    one-launch LDS sweep gives the same bits as one launch per colour, for
    every level of a full-mode solve (patch 1 wrapping the periodic domain in
    one case), and the oracle's answer."""
    say(f"patch fused sweep m={m} pn2={pn2} wrap={wrap}")
    n = max(64, m // 2)
    f = synth.make_field(n, 2.0, 51, n_tophats=8)
    c = synth.densest_tophat_centre(f)
    o1 = synth.patch_origin_centred(c, m // 2)
    if wrap:
        o1 = (-m // 8, o1[1], o1[2])
    c1 = tuple((c[a] - o1[a]) * 2 for a in range(3))
    o2 = tuple(min(max(v, 8), m - pn2 // 2 - 8) for v in synth.patch_origin_centred(c1, pn2 // 2))
    d1 = synth.patch_delta(f, n, [o1], m)
    d2 = synth.patch_delta(f, n, [o1, o2], pn2)
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n),
                     patches=[ndgp.Patch(m, o1), ndgp.Patch(pn2, o2)])
    deltas = [dev(x) for x in (f.delta, d1, d2)]
    p = dict(rc=1.0, tol=0.0, max_cycles=200)
    a, ra = ndgp.solve(grid, ndgp.Params(**p), deltas)
    b, rb = ndgp.solve(grid, ndgp.Params(two_pass=True, **p), deltas)
    torch.cuda.synchronize()
    say(f"  cycles={ra.cycles} rel_res={ra.rel_res}")
    assert ra.status == 0 and ra.cycles == rb.cycles
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    if m == 128 and not wrap:
        beta = O.beta_lcdm(1.0, 0.3, 1.0)
        prob = O.Problem(delta=[f.delta, d1, d2], h=grid.h, rc=1.0, beta=beta, origins=(o1, o2))
        phio, infos = O.solve_problem(prob)
        for lvl in range(3):
            e = rel(a[lvl].cpu().numpy(), phio[lvl])
            say(f"  level {lvl}: rel err {e:.2e}")
            assert e <= PHI_TOL


@pytest.mark.parametrize("m,depth,cellwise", [(32, 2, False), (64, 2, False), (16, 2, False),
                                               (32, 2, True), (64, 1, True), (128, 1, True),
                                               (256, 1, True)])
def test_patch_bottom_bitwise_equal_per_level_launches(m, depth, cellwise):
    """The coarse levels of a refinement from 16^3 down (ghost shells that
    follow the interior, held cells of the cell-wise mode) solved in one
    workgroup, and 128^3 and 256^3 refinements with held cells relaxed by the
    one-launch LDS sweep (held cells kept, workgroups of held cells skipped;
    chunks of 4 and of 32 planes), give the
    same bits, cycle counts and event counts as one launch per colour, per
    transfer and per level (patches of 16^3 have no such levels: both paths
    are the per-level launches)."""
    say(f"patch bottom m={m} depth={depth} cellwise={cellwise}")
    f, deltas, grid = deep_patch_problem(n=max(32, m), m=m, depth=depth, seed=14)
    dd = [dev(d) for d in deltas]
    p = dict(rc=1.0, tol=0.0, max_cycles=200)
    if not cellwise:
        a, ra = ndgp.solve(grid, ndgp.Params(**p), dd)
        b, rb = ndgp.solve(grid, ndgp.Params(two_pass=True, **p), dd)
    else:
        beta = ndgp.beta_lcdm(1.0, 0.3, 1.0)
        psi = ndgp.solve(grid, ndgp.Params(rc=0.0, beta=beta, tol=0.0, max_cycles=200), dd)[0]
        psi = [1.5 * beta * x for x in psi]
        for thr in (0.12, 0.11, 0.13, 0.1, 0.14, 0.09, 0.15, 0.08, 0.06):
            a, ra = ndgp.solve_cellwise(grid, ndgp.Params(**p), dd, psi, thr)
            if 0.05 < ra.iterated_fraction[1] < 0.95:
                break
        say(f"  threshold {thr}: iterated {ra.iterated_fraction[:depth + 1]}")
        assert 0.05 < ra.iterated_fraction[1] < 0.95
        b, rb = ndgp.solve_cellwise(grid, ndgp.Params(two_pass=True, **p), dd, psi, thr)
    torch.cuda.synchronize()
    say(f"  cycles={ra.cycles} rel_res={ra.rel_res}")
    assert ra.status == 0 and rb.status == 0
    assert ra.cycles == rb.cycles and ra.fallbacks == rb.fallbacks and ra.holds == rb.holds
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("nu1,nu2", [(1, 1), (3, 1), (1, 3)])
def test_odd_sweep_counts(nu1, nu2):
    """Odd numbers of pre/post sweeps: the fused one-launch sweeps take the
    even part and per-colour launches the last sweep, and the first post
    sweep still adds the coarse correction.  Same bits as per-level
    launches, and the oracle's answer with the same sweep counts."""
    say(f"odd sweeps nu1={nu1} nu2={nu2}")
    n, h, rc = 128, ndgp.cell_size(128.0, 128), 1.0
    f = synth.make_field(n, 2.0, 41, n_tophats=10)
    d = dev(f.delta)
    grid = ndgp.Grid(n=n, h=h)
    p = dict(rc=rc, tol=0.0, max_cycles=200, nu1=nu1, nu2=nu2)
    a, ra = ndgp.solve(grid, ndgp.Params(**p), [d])
    b, rb = ndgp.solve(grid, ndgp.Params(two_pass=True, **p), [d])
    torch.cuda.synchronize()
    assert ra.status == 0 and ra.cycles == rb.cycles and ra.history == rb.history
    assert torch.equal(a[0], b[0])
    beta = O.beta_lcdm(1.0, 0.3, rc)
    S, _ = O.source(f.delta, 0.3, 1.0, beta)
    phio, info = O.solve_periodic(S, h, O.alpha(rc, beta, 1.0), nu1=nu1, nu2=nu2)
    assert info.status == 0
    assert rel(a[0].cpu().numpy(), phio) <= PHI_TOL


@pytest.mark.parametrize("n", [128, 256])
def test_fused_corr_sweep_bitwise_equals_per_colour_launches(n):
    """Mixed precision: the one-launch LDS sweep of the FP32 correction gives
    the same bits for the whole solve as one k_corr_half launch per colour."""
    say(f"mixed fused vs per-colour n={n}")
    f = synth.make_field(n, 2.0, 37, n_tophats=10)
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n))
    d = dev(f.delta)
    p = dict(rc=1.0, tol=1e-10, precision=ndgp.PREC_MIXED)
    a, ra = ndgp.solve(grid, ndgp.Params(**p), [d])
    b, rb = ndgp.solve(grid, ndgp.Params(two_pass=True, **p), [d])
    torch.cuda.synchronize()
    assert ra.cycles == rb.cycles and ra.history == rb.history
    assert torch.equal(a[0], b[0])


MIXED_TOL = 1e-8


@pytest.mark.parametrize("rc", [0.5, 1.0, 5.0])
def test_mixed_precision_matches_oracle(rc):
    """FP32 multigrid on the correction inside the FP64 defect-correction loop
    reaches the FP64 oracle's answer within the mixed-precision bar."""
    n = 64
    say(f"mixed n={n} rc={rc}")
    f = synth.make_field(n, 2.5, 40, n_tophats=4)
    h = ndgp.cell_size(128.0, n)
    phio, S = oracle_periodic(f.delta, h, rc)
    (phig,), rep = gpu_solve([f.delta], ndgp.Grid(n=n, h=h), rc=rc, tol=1e-12, max_cycles=100,
                             precision=ndgp.PREC_MIXED)
    say(f"  outer={rep.cycles[0]} rel_res={rep.rel_res[0]:.2e} hist={[f'{x:.1e}' for x in rep.history]}")
    assert rep.status == 0
    assert rel(phig, phio) <= MIXED_TOL


def test_warm_start_and_errors():
    n = 32
    f = synth.make_field(n, 1.0, 1512)
    h = ndgp.cell_size(64.0, n)
    grid = ndgp.Grid(n=n, h=h)
    say("warm start")
    phi, rep = ndgp.solve(grid, ndgp.Params(rc=1.0, tol=1e-10), [dev(f.delta)])
    phi2, rep2 = ndgp.solve(grid, ndgp.Params(rc=1.0, tol=1e-10, warm_start=True), [dev(f.delta)],
                            phi=[phi[0].clone()])
    assert rep2.cycles[0] == 0
    say("no convergence")
    _, rep3 = ndgp.solve(grid, ndgp.Params(rc=1.0, tol=1e-14, max_cycles=2), [dev(f.delta)],
                         check=False)
    assert rep3.status == ndgp.NDGP_ENOCONV and rep3.cycles[0] == 2
    say("non-finite delta")
    bad = f.delta.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(ndgp.NdgpError) as e:
        ndgp.solve(grid, ndgp.Params(rc=1.0), [dev(bad)])
    assert e.value.status == ndgp.NDGP_EINVAL
    say("workspace too small")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ndgp.NdgpError) as e:
        ndgp.solve(grid, ndgp.Params(rc=1.0), [dev(f.delta)], ws=small)
    assert e.value.status == ndgp.NDGP_ENOMEM


# --------------------------------------------------------------------------
# refined patches (Sec. III.A) and the interpolated mode (Sec. III.B)

def patch_problem(n=64, pn=(64, 64), seed=11, wrap=False):
    f = synth.make_field(n, 2.0, seed, n_tophats=10)
    c = synth.densest_tophat_centre(f)
    o1 = synth.patch_origin_centred(c, pn[0] // 2)
    if wrap:
        o1 = (-pn[0] // 8, o1[1], o1[2])  # patch 1 straddles the periodic boundary
    c1 = tuple((c[a] - o1[a]) * 2 for a in range(3))
    o2 = synth.patch_origin_centred(c1, pn[1] // 2)
    o2 = tuple(min(max(v, 8), pn[0] - pn[1] // 2 - 8) for v in o2)
    d1 = synth.patch_delta(f, n, [o1], pn[0])
    d2 = synth.patch_delta(f, n, [o1, o2], pn[1])
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n),
                     patches=[ndgp.Patch(pn[0], o1), ndgp.Patch(pn[1], o2)])
    return f, [f.delta, d1, d2], grid


@pytest.mark.parametrize("interpolated", [False, True])
@pytest.mark.parametrize("wrap", [False, True])
def test_patches_match_oracle(interpolated, wrap):
    say(f"patches interpolated={interpolated} wrap={wrap}")
    rc = 1.0
    f, deltas, grid = patch_problem(wrap=wrap)
    beta = O.beta_lcdm(1.0, 0.3, rc)
    prob = O.Problem(delta=deltas, h=grid.h, rc=rc, beta=beta,
                     origins=tuple(p.origin for p in grid.patches))
    phio, infos = O.solve_problem(prob, interpolated=interpolated)
    for inf in infos[: (1 if interpolated else 3)]:
        assert inf.status == 0
    mode = ndgp.MODE_INTERPOLATED if interpolated else ndgp.MODE_FULL
    phig, rep = gpu_solve(deltas, grid, rc=rc, tol=0.0, max_cycles=200, mode=mode)
    say(f"  cycles={rep.cycles} rel_res={rep.rel_res}")
    assert rep.status == 0
    for lvl in range(3):
        e = rel(phig[lvl], phio[lvl])
        say(f"  level {lvl}: rel err {e:.2e}")
        assert e <= PHI_TOL
    # forces from the same fields agree to rounding; end to end within the bar
    fg = [x.cpu().numpy() for x in ndgp.force(grid, [dev(p) for p in phig])]
    for lvl in range(3):
        fo = O.force(phig[lvl], grid.level_h(lvl), periodic=(lvl == 0))
        assert np.abs(fg[lvl] - fo).max() <= 1e-13 * np.abs(fo).max()
        fo_or = O.force(phio[lvl], grid.level_h(lvl), periodic=(lvl == 0))
        assert rel(fg[lvl], fo_or) <= 1e-10


@pytest.mark.parametrize("interpolated", [False, True])
def test_mixed_precision_with_patches_matches_oracle(interpolated):
    """Mixed precision on the domain (FP32 correction multigrid) with two
    nested refinements relaxed in FP64 from ghost shells of that domain
    solution (full mode), or interpolated from it: every level within the
    mixed-precision bar of the FP64 oracle."""
    say(f"mixed + patches interpolated={interpolated}")
    rc = 1.0
    f, deltas, grid = patch_problem()
    beta = O.beta_lcdm(1.0, 0.3, rc)
    prob = O.Problem(delta=deltas, h=grid.h, rc=rc, beta=beta,
                     origins=tuple(p.origin for p in grid.patches))
    phio, infos = O.solve_problem(prob, interpolated=interpolated)
    mode = ndgp.MODE_INTERPOLATED if interpolated else ndgp.MODE_FULL
    phig, rep = gpu_solve(deltas, grid, rc=rc, tol=1e-12, max_cycles=200, mode=mode,
                          precision=ndgp.PREC_MIXED)
    say(f"  cycles={rep.cycles} rel_res={rep.rel_res}")
    assert rep.status == 0
    for lvl in range(3):
        e = rel(phig[lvl], phio[lvl])
        say(f"  level {lvl}: rel err {e:.2e}")
        assert e <= MIXED_TOL


def deep_patch_problem(n=32, m=32, depth=4, seed=12):
    """``depth`` nested patches of m cells (ratio 2 each), centred on the
    largest top-hat and kept 2 parent cells inside their parent."""
    f = synth.make_field(n, 2.0, seed, n_tophats=6)
    c = synth.densest_tophat_centre(f)
    chain, deltas, patches = [], [f.delta], []
    for q in range(depth):
        o = synth.patch_origin_centred(c, m // 2)
        if q > 0:
            o = tuple(min(max(v, 2), m - m // 2 - 2) for v in o)
        chain.append(o)
        deltas.append(synth.patch_delta(f, n, chain, m))
        patches.append(ndgp.Patch(m, o))
        c = tuple((c[a] - o[a]) * 2 for a in range(3))
    return f, deltas, ndgp.Grid(n=n, h=ndgp.cell_size(float(n), n), patches=patches)


@pytest.mark.parametrize("trunc", [1, 2, 3, 4, 5])
def test_truncation_levels_match_oracle(trunc):
    """NDGP_MODE_TRUNCATED on four nested patches (Sec. IV.A, l_trunc =
    l_d + trunc): the relaxed levels are those of the full mode bit for bit,
    the truncated ones are interpolated from their own parent, and every level
    matches the oracle's truncated path."""
    say(f"truncation level {trunc}: 32^3 + 4 nested 32^3 patches")
    rc = 1.0
    f, deltas, grid = deep_patch_problem()
    beta = O.beta_lcdm(1.0, 0.3, rc)
    prob = O.Problem(delta=deltas, h=grid.h, rc=rc, beta=beta,
                     origins=tuple(p.origin for p in grid.patches))
    phio, infos = O.solve_problem(prob, trunc_level=trunc)
    for inf in infos[:trunc]:
        assert inf.status == 0
    phit, rept = gpu_solve(deltas, grid, rc=rc, tol=0.0, max_cycles=200,
                           mode=ndgp.MODE_TRUNCATED, trunc_level=trunc)
    say(f"  cycles={rept.cycles} rel_res={rept.rel_res}")
    assert rept.status == 0
    phif, repf = gpu_solve(deltas, grid, rc=rc, tol=0.0, max_cycles=200, mode=ndgp.MODE_FULL)
    for lvl in range(5):
        e = rel(phit[lvl], phio[lvl])
        say(f"  level {lvl}: rel err {e:.2e}")
        assert e <= PHI_TOL
        if lvl < trunc:
            assert np.array_equal(phit[lvl], phif[lvl])
            assert rept.cycles[lvl] == repf.cycles[lvl] and rept.rel_res[lvl] >= 0.0
        else:
            assert rept.cycles[lvl] == 0 and rept.rel_res[lvl] == -1.0
            pq = grid.patches[lvl - 1]
            want = O.interpolate(phit[lvl - 1], lvl == 1, pq.origin, 0, pq.n)
            assert np.abs(phit[lvl] - want).max() <= 1e-14 * np.abs(want).max()
    fg = [x.cpu().numpy() for x in ndgp.force(grid, [dev(p) for p in phit])]
    for lvl in range(5):
        fo = O.force(phio[lvl], grid.level_h(lvl), periodic=(lvl == 0))
        assert rel(fg[lvl], fo) <= 1e-10


def _parent_ratio(phi_par, psi_par, periodic, origin, nc):
    """|F_5th| / |F_GR| = |grad phi| / (2 |grad psi|) at the parent cell of every
    child cell (numpy, from the oracle's own fields)."""
    idx = [origin[a] + np.arange(nc) // 2 for a in range(3)]
    g_phi, g_psi = 0.0, 0.0
    for a in range(3):
        up = [ix.copy() for ix in idx]
        dn = [ix.copy() for ix in idx]
        up[a] = up[a] + 1
        dn[a] = dn[a] - 1

        def take(f, q):
            if periodic:
                n = f.shape[0]
                return f[np.ix_(q[2] % n, q[1] % n, q[0] % n)]
            return f[np.ix_(q[2] + 1, q[1] + 1, q[0] + 1)]
        g_phi = g_phi + (take(phi_par, up) - take(phi_par, dn)) ** 2
        g_psi = g_psi + (take(psi_par, up) - take(psi_par, dn)) ** 2
    return np.sqrt(g_phi) / (2.0 * np.sqrt(g_psi))


def test_cellwise_truncation_matches_oracle():
    """ndgp_solve_cellwise (Sec. III.C) on a 32^3 domain with two nested 32^3
    patches, the Newtonian potential from each side's own r_c = 0 solve: the
    iterated cells are the oracle's exactly and every level matches the
    oracle's masked solve.  Threshold 0 is ndgp_solve bit for bit, an infinite
    one the interpolated mode bit for bit."""
    rc = 1.0
    f, deltas, grid = deep_patch_problem(depth=2)
    beta = O.beta_lcdm(1.0, 0.3, rc)
    origins = tuple(p.origin for p in grid.patches)
    say("cellwise: oracle r_c = 0 and full solves")
    lin = O.Problem(delta=deltas, h=grid.h, rc=0.0, beta=beta, origins=origins)
    psi_o = [1.5 * beta * p for p in O.solve_problem(lin)[0]]
    prob = O.Problem(delta=deltas, h=grid.h, rc=rc, beta=beta, origins=origins)
    full_o, _ = O.solve_problem(prob)
    # a threshold whose nearest parent ratio is far from it on both levels
    r1 = np.sort(_parent_ratio(full_o[0], psi_o[0], True, origins[0], 32).ravel())
    chosen = None
    for qtl in (0.5, 0.4, 0.6, 0.3, 0.7):
        k = int(qtl * (len(r1) - 1))
        gaps = np.diff(r1[k - 50:k + 50])
        g = int(np.argmax(gaps))
        thr = 0.5 * (r1[k - 50 + g] + r1[k - 50 + g + 1])
        phio, infos, masks = O.solve_problem(prob, cellwise=(psi_o, thr))
        r2 = _parent_ratio(phio[1], psi_o[1], False, origins[1], 32)
        m1 = np.min(np.abs(r1 / thr - 1.0))
        m2 = np.min(np.abs(r2 / thr - 1.0))
        if min(m1, m2) > 1e-7 and all(i.status == 0 for i in infos):
            chosen = thr
            break
    assert chosen is not None
    say(f"  threshold {chosen:.6g}: iterated {[int(mk.sum()) for mk in masks[1:]]} of {32**3}")
    psi_g = ndgp.solve(grid, ndgp.Params(rc=0.0, beta=beta, tol=0.0, max_cycles=200),
                       [dev(d) for d in deltas])[0]
    psi_g = [1.5 * beta * p for p in psi_g]
    params = ndgp.Params(rc=rc, tol=0.0, max_cycles=200)
    phig, rep = ndgp.solve_cellwise(grid, params, [dev(d) for d in deltas], psi_g, chosen)
    torch.cuda.synchronize()
    say(f"  cycles={rep.cycles} iterated={rep.iterated_fraction[:3]}")
    assert rep.status == 0
    for lvl in (1, 2):
        assert rep.iterated_fraction[lvl] == masks[lvl].sum() / 32**3
        assert 0.0 < rep.iterated_fraction[lvl] < 1.0
    for lvl in range(3):
        e = rel(phig[lvl].cpu().numpy(), phio[lvl])
        say(f"  level {lvl}: rel err {e:.2e}")
        assert e <= PHI_TOL
    # held cells keep exactly the interpolated value of the GPU's own parent
    for lvl in (1, 2):
        pq = grid.patches[lvl - 1]
        want = O.interpolate(phig[lvl - 1].cpu().numpy(), lvl == 1, pq.origin, 0, pq.n)
        held = masks[lvl] == 0
        got = phig[lvl].cpu().numpy()[1:-1, 1:-1, 1:-1][held]
        assert np.abs(got - want[1:-1, 1:-1, 1:-1][held]).max() <= 1e-14 * np.abs(want).max()
    # with a truncation level: patch 1 cell-wise, patch 2 interpolated from it
    phot, _, mkt = O.solve_problem(prob, cellwise=(psi_o, chosen), trunc_level=2)
    pt = ndgp.Params(rc=rc, tol=0.0, max_cycles=200, mode=ndgp.MODE_TRUNCATED, trunc_level=2)
    phgt, rept = ndgp.solve_cellwise(grid, pt, [dev(d) for d in deltas], psi_g, chosen)
    assert rept.status == 0 and rept.iterated_fraction[2] == 0.0 and rept.cycles[2] == 0
    assert rept.iterated_fraction[1] == mkt[1].sum() / 32**3
    for lvl in range(3):
        assert rel(phgt[lvl].cpu().numpy(), phot[lvl]) <= PHI_TOL
    # the limits, bit for bit
    dd = [dev(d) for d in deltas]
    ph0, r0 = ndgp.solve_cellwise(grid, params, dd, psi_g, 0.0)
    phf, rf = ndgp.solve(grid, params, dd)
    phinf, _ = ndgp.solve_cellwise(grid, params, dd, psi_g, float("inf"))
    phi_i, _ = ndgp.solve(grid, ndgp.Params(rc=rc, tol=0.0, max_cycles=200,
                                            mode=ndgp.MODE_INTERPOLATED), dd)
    for lvl in range(3):
        assert torch.equal(ph0[lvl], phf[lvl])
        assert torch.equal(phinf[lvl], phi_i[lvl])
    assert r0.cycles == rf.cycles and r0.iterated_fraction[:3] == [1.0, 1.0, 1.0]


@pytest.mark.parametrize("n", [64, 128, 256])
def test_force_matches_oracle_on_periodic_levels(n):
    """F5 on a periodic level (Sec. III.B): the z-streamed kernel (n >= 128)
    and the per-cell kernel (64^3) against the oracle's central differences
    of the same field, with the wrap-around cells of every face."""
    rng = np.random.default_rng(900 + n)
    phi = rng.standard_normal((n, n, n))
    h = ndgp.cell_size(256.0, n)
    grid = ndgp.Grid(n=n, h=h)
    say(f"[force] n={n}")
    fg = ndgp.force(grid, [dev(phi)])[0].cpu().numpy()
    fo = O.force(phi, h, periodic=True)
    assert fg.shape == fo.shape
    assert np.abs(fg - fo).max() <= 1e-13 * np.abs(fo).max()


def test_total_force_and_geff_stats_match_oracle():
    """ndgp_total_force and ndgp_geff_stats (Eq. modpoisson, Sec. III.B; the
    per-level G_eff of Fig. 3 over cells) on seeded fields: a 32^3 domain and
    two nested 32^3 patches, one wrapping the periodic domain.  Identical
    inputs give identical per-cell ratios, so cell counts, histograms, min and
    max agree exactly and the sums to rounding."""
    from oracle import geff as G
    f, deltas, grid = deep_patch_problem(depth=2)
    rng = np.random.default_rng(77)
    phis, psis = [], []
    for lvl in range(3):
        m = grid.level_n(lvl)
        a = synth.make_field(m, 1.0, 300 + lvl).delta
        b = synth.make_field(m, 1.0, 400 + lvl).delta * 3.0 + 0.5 * a
        if lvl:  # patches: padded fields with arbitrary ghost values
            a = np.pad(a, 1, mode="wrap") + 1e-3 * rng.standard_normal((m + 2,) * 3)
            b = np.pad(b, 1, mode="wrap")
        phis.append(a)
        psis.append(b)
    edges = np.geomspace(1e-3, 10.0, 41)
    got, hist = ndgp.geff_stats(grid, [dev(x) for x in phis], [dev(x) for x in psis], edges)
    want, hist_o = G.geff_stats(phis, psis, [p.origin for p in grid.patches],
                                [p.n for p in grid.patches], edges)
    np.testing.assert_array_equal(hist, hist_o)
    for lvl in range(3):
        say(f"  level {lvl}: {got[lvl]['cells']} cells, mean G_eff-1 {got[lvl]['mean']:.4f}")
        assert got[lvl]["cells"] == want[lvl]["cells"] == hist[lvl].sum()
        assert got[lvl]["min"] == want[lvl]["min"] and got[lvl]["max"] == want[lvl]["max"]
        assert got[lvl]["sum"] == pytest.approx(want[lvl]["sum"], rel=1e-12)
        assert got[lvl]["sum_sq"] == pytest.approx(want[lvl]["sum_sq"], rel=1e-12)
    assert got[0]["cells"] == 32**3 - 16**3 and got[2]["cells"] == 32**3
    F = ndgp.total_force(grid, [dev(x) for x in phis], [dev(x) for x in psis])
    for lvl in range(3):
        Fo = G.total_force(phis[lvl], psis[lvl], grid.level_h(lvl), lvl == 0)
        Fg = F[lvl].cpu().numpy()
        assert np.abs(Fg - Fo).max() <= 1e-13 * np.abs(Fo).max()
    with pytest.raises(ndgp.NdgpError):
        ndgp.geff_stats(grid, [dev(x) for x in phis], [dev(x) for x in psis], edges[::-1])


def test_patch_residual_level():
    """ndgp_residual on a patch level uses the ghost shell as boundary."""
    f, deltas, grid = patch_problem()
    phig, rep = gpu_solve(deltas, grid, rc=1.0, tol=1e-10)
    beta = O.beta_lcdm(1.0, 0.3, 1.0)
    al = O.alpha(1.0, beta, 1.0)
    _, mean = O.source(deltas[0], 0.3, 1.0, beta)
    for lvl in (1, 2):
        say(f"patch residual level {lvl}")
        S = O.source_shift(deltas[lvl], mean, 0.3, 1.0, beta)
        ro = S - O.operator_padded(phig[lvl], grid.level_h(lvl), al)
        r, relg = ndgp.residual(grid, ndgp.Params(rc=1.0), [dev(d) for d in deltas],
                                dev(phig[lvl]), level=lvl)
        assert np.abs(r.cpu().numpy() - ro).max() <= 1e-12 * np.abs(S).max()
        assert relg <= 1e-10


# --------------------------------------------------------------------------
# full sizes, in the launch configuration the benchmark times

@pytest.mark.parametrize("n,box,sigma,tophats,rc,seed,prec", [
    (256, 256.0, 2.0, 50, 1.0, 1513, ndgp.PREC_FP64),   # 256^3 lognormal + 50 top-hats
    (512, 512.0, 2.5, 0, 1.0, 1515, ndgp.PREC_FP64),    # 512^3 lognormal, sigma 2.5
    (512, 512.0, 2.5, 0, 5.0, 1515, ndgp.PREC_MIXED),   # same, mixed precision, r_c = 5
])
def test_full_size_residual_by_oracle(n, box, sigma, tophats, rc, seed, prec):
    say(f"full size n={n} precision={prec}: generating")
    f = synth.make_field(n, sigma, seed, n_tophats=tophats)
    h = ndgp.cell_size(box, n)
    grid = ndgp.Grid(n=n, h=h)
    params = ndgp.Params(rc=rc, tol=1e-10, precision=prec)
    d = dev(f.delta)
    say(f"full size n={n}: solving")
    phi, rep = ndgp.solve(grid, params, [d])
    r, relg = ndgp.residual(grid, params, [d], phi[0])
    torch.cuda.synchronize()
    say(f"  cycles={rep.cycles[0]} rel_res={rep.rel_res[0]:.3e} t={rep.t_total_ms:.1f} ms")
    assert rep.status == 0 and rep.rel_res[0] <= 1e-10
    phig = phi[0].cpu().numpy()
    rg = r.cpu().numpy()
    del phi, r, d
    beta = O.beta_lcdm(1.0, 0.3, rc)
    al = O.alpha(rc, beta, 1.0)
    S, _ = O.source(f.delta, 0.3, 1.0, beta)
    rng = np.random.default_rng(0)
    cells = rng.integers(0, n, size=(4096, 3))
    cells[:8] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 0], [n - 1, 0, n - 1],
                 [n // 2, 0, n - 1], [1, 1, 1], [n - 2, n - 1, 0], [0, 0, n - 1]]
    ro = S[cells[:, 2], cells[:, 1], cells[:, 0]] - O.operator_at(phig, h, al, cells)
    scale = np.abs(S).max()
    assert np.abs(rg[cells[:, 2], cells[:, 1], cells[:, 0]] - ro).max() <= 1e-12 * scale
    say(f"full size n={n}: oracle residual over the whole grid")
    del rg
    ro_all = S - O.operator(phig, h, al)
    assert np.linalg.norm(ro_all) / np.linalg.norm(S) == pytest.approx(relg, rel=1e-6)
    assert relg <= 1e-10


def test_full_size_patches_by_oracle():
    """The benchmark's patch configuration at full size: 256^3 lognormal
    sigma 2 + 50 top-hats, two nested 128^3 patches at 2x and 4x centred on
    the largest top-hat.  Full mode: each patch's ghost shell is the oracle's
    trilinear interpolation of its converged parent, and its residual (from
    that shell) is the oracle's over the whole patch, below the tolerance.
    Interpolated mode: each patch, interior and ghosts, is the oracle's
    interpolation of its GPU parent."""
    n, box, rc, m = 256, 256.0, 1.0, 128
    say("full-size patches: generating")
    f = synth.make_field(n, 2.0, 1513, n_tophats=50)
    c = synth.densest_tophat_centre(f)
    chain, deltas, patches = [], [f.delta], []
    for q in range(2):
        o = synth.patch_origin_centred(c, m // 2)
        if q > 0:
            o = tuple(min(max(v, 8), m - m // 2 - 8) for v in o)
        chain.append(o)
        deltas.append(synth.patch_delta(f, n, chain, m))
        patches.append(ndgp.Patch(m, o))
        c = tuple((c[a] - o[a]) * 2 for a in range(3))
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(box, n), patches=patches)
    beta = O.beta_lcdm(1.0, 0.3, rc)
    al = O.alpha(rc, beta, 1.0)
    _, mean = O.source(deltas[0], 0.3, 1.0, beta)
    shell = np.ones((m + 2,) * 3, dtype=bool)
    shell[1:-1, 1:-1, 1:-1] = False
    for mode in (ndgp.MODE_FULL, ndgp.MODE_INTERPOLATED):
        say(f"full-size patches: mode {mode}")
        phig, rep = gpu_solve(deltas, grid, rc=rc, tol=1e-10, mode=mode)
        assert rep.status == 0 and rep.rel_res[0] <= 1e-10
        for lvl in (1, 2):
            want = O.interpolate(phig[lvl - 1], lvl == 1, chain[lvl - 1], 0, m)
            scale = np.abs(want).max()
            if mode == ndgp.MODE_INTERPOLATED:
                assert np.abs(phig[lvl] - want).max() <= 1e-14 * scale
                continue
            assert np.abs(phig[lvl][shell] - want[shell]).max() <= 1e-14 * scale
            S = O.source_shift(deltas[lvl], mean, 0.3, 1.0, beta)
            ro = S - O.operator_padded(phig[lvl], grid.level_h(lvl), al)
            r, relg = ndgp.residual(grid, ndgp.Params(rc=rc), [dev(d) for d in deltas],
                                    dev(phig[lvl]), level=lvl)
            say(f"  level {lvl}: cycles={rep.cycles[lvl]} rel_res={relg:.2e}")
            assert np.abs(r.cpu().numpy() - ro).max() <= 1e-12 * np.abs(S).max()
            assert relg <= 1e-10 and rep.rel_res[lvl] <= 1e-10


def test_largest_grid_sampled_residual():
    """n = 1024, the largest grid the library takes (about 35 GB of device
    memory with the workspace): lognormal sigma 2.5 drawn on the device, FP64
    to 1e-10; the oracle's residual at 4096 sampled cells (boundary corners
    included) equals the GPU residual there."""
    n, box, rc = 1024, 1024.0, 1.0
    say("largest grid n=1024: generating on the device")
    d = synth.lognormal_delta_torch(n, 2.5, 1516)
    h = ndgp.cell_size(box, n)
    grid = ndgp.Grid(n=n, h=h)
    params = ndgp.Params(rc=rc, tol=1e-10)
    say("largest grid n=1024: solving")
    phi, rep = ndgp.solve(grid, params, [d])
    r, relg = ndgp.residual(grid, params, [d], phi[0])
    torch.cuda.synchronize()
    say(f"  cycles={rep.cycles[0]} rel_res={rep.rel_res[0]:.3e} t={rep.t_total_ms:.1f} ms")
    assert rep.status == 0 and rep.rel_res[0] <= 1e-10 and relg <= 1e-10
    rng = np.random.default_rng(1)
    cells = rng.integers(0, n, size=(4096, 3))
    cells[:4] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 0], [n - 1, 0, n - 1]]
    idx = torch.from_numpy(cells).to("cuda")
    rg = r[idx[:, 2], idx[:, 1], idx[:, 0]].cpu().numpy()
    del r
    say("largest grid n=1024: oracle residual at sampled cells")
    phig = phi[0].cpu().numpy()
    del phi
    delta = d.cpu().numpy()
    del d
    torch.cuda.empty_cache()
    beta = O.beta_lcdm(1.0, 0.3, rc)
    S, _ = O.source(delta, 0.3, 1.0, beta)
    del delta
    ro = S[cells[:, 2], cells[:, 1], cells[:, 0]] - O.operator_at(phig, h, O.alpha(rc, beta, 1.0),
                                                                  cells)
    assert np.abs(rg - ro).max() <= 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("prec,damped", [(ndgp.PREC_FP64, False), (ndgp.PREC_MIXED, False),
                                         (ndgp.PREC_FP64, True), (ndgp.PREC_MIXED, True)])
def test_extreme_source_matches_oracle(prec, damped):
    """A lognormal field with sigma_ln 2.47 (delta up to ~1e5 in one cell) at
    r_cH0 = 5 on 1 Mpc/h cells.  Holding cells past the vertex of their
    quadratic made these cycles diverge after reaching 1e-3; with the root on
    the elliptic side they converge with the plain step (no safeguard restart),
    and with the damped step u + 0.8 du from the start (NDGP_DAMPED, the mode
    the safeguard restarts in).  phi at the 1e-10 tolerance is the oracle's
    (run to 1e-12) within the 1e-8 bar."""
    n, rc, sigma, seed = 256, 5.0, 2.4694042826895837, 100881
    say(f"extreme source n={n} rc={rc} precision={prec} damped={damped}")
    d = synth.lognormal_delta_torch(n, sigma, seed, device="cuda")
    h = ndgp.cell_size(float(n), n)
    phi, rep = ndgp.solve(ndgp.Grid(n=n, h=h),
                          ndgp.Params(rc=rc, tol=1e-10, precision=prec, max_cycles=60,
                                      damped=damped), [d])
    torch.cuda.synchronize()
    say(f"  cycles={rep.cycles[0]} damped_from={rep.damped_from[0]} holds={rep.holds} "
        f"hist={[f'{x:.1e}' for x in rep.history]}")
    assert rep.status == 0 and rep.rel_res[0] <= 1e-10
    assert rep.damped_from[0] == (1 if damped else 0)
    key = ("extreme", n, seed)
    if key not in _oracle_cache:
        _oracle_cache.clear()
        dn = d.cpu().numpy()
        beta = O.beta_lcdm(1.0, 0.3, rc)
        S, _ = O.source(dn, 0.3, 1.0, beta)
        phio, info = O.solve_periodic(S, h, O.alpha(rc, beta, 1.0), tol=1e-12)
        say(f"  oracle: {info.cycles} cycles, rel_res {info.rel_res:.2e}")
        assert info.status == 0
        _oracle_cache[key] = phio
    e = rel(phi[0].cpu().numpy(), _oracle_cache[key])
    say(f"  rel err vs oracle {e:.2e}")
    assert e <= MIXED_TOL


_oracle_cache = {}


# --------------------------------------------------------------------------
# the branches of the per-cell root (Sec. III.A, Eq. newton)

@pytest.mark.parametrize("prec", [ndgp.PREC_FP64, ndgp.PREC_MIXED])
def test_cells_past_their_vertex_take_the_elliptic_root_and_match_oracle(prec):
    """A warm start far from the answer (white noise of 1.6e-8 on 1 Mpc/h
    cells at r_cH0 = 5) puts about 10% of the cells past the vertex of their
    own quadratic on the first visit (dL/dphi of the cell equation has the
    non-elliptic sign there); those cells move to the root on the elliptic
    side.  The solve reaches the unique elliptic solution, the oracle's from
    its own nested start."""
    n, rc = 32, 5.0
    say(f"past-vertex cells precision={prec}")
    f = synth.make_field(n, 2.0, 61, n_tophats=4)
    h = ndgp.cell_size(32.0, n)
    phio, _ = oracle_periodic(f.delta, h, rc)
    rng = np.random.default_rng(7)
    phi0 = dev(1.6e-8 * rng.standard_normal((n, n, n)))
    grid = ndgp.Grid(n=n, h=h)
    tol = 0.0 if prec == ndgp.PREC_FP64 else 1e-12
    phi, rep = ndgp.solve(grid, ndgp.Params(rc=rc, tol=tol, max_cycles=200, precision=prec,
                                            warm_start=True), [dev(f.delta)], phi=[phi0])
    torch.cuda.synchronize()
    say(f"  cycles={rep.cycles[0]} holds={rep.holds} fallbacks={rep.fallbacks} "
        f"damped_from={rep.damped_from[0]} rel_res={rep.rel_res[0]:.2e}")
    assert rep.status == 0
    assert rep.holds > 0
    e = rel(phi[0].cpu().numpy(), phio)
    say(f"  rel err vs oracle {e:.2e}")
    assert e <= (PHI_TOL if prec == ndgp.PREC_FP64 else MIXED_TOL)


@pytest.mark.parametrize("prec", [ndgp.PREC_FP64, ndgp.PREC_MIXED])
def test_no_real_root_on_an_unphysical_void(prec):
    """The cell quadratic has no real root only where alpha S < -3/8, i.e.
    delta far below -1 (an oracle pin shows this bound); there the
    relaxation moves the cell to the vertex of its quadratic and counts the
    event.  Three cells at delta = -40 (r_cH0 = 5): no elliptic solution exists
    near them, the oracle fails too, and the solve ends with NDGP_ENOCONV after
    counting the no-root visits instead of hanging or faulting."""
    n, rc = 32, 5.0
    say(f"unphysical void precision={prec}")
    f = synth.make_field(n, 2.0, 61, n_tophats=4)
    d = f.delta.copy()
    for (i, j, k) in ((5, 6, 7), (20, 21, 3), (11, 27, 30)):
        d[k, j, i] = -40.0
    h = ndgp.cell_size(32.0, n)
    beta = O.beta_lcdm(1.0, 0.3, rc)
    S, _ = O.source(d, 0.3, 1.0, beta)
    assert O.alpha(rc, beta, 1.0) * S.min() < -3 / 8
    _, info = O.solve_periodic(S, h, O.alpha(rc, beta, 1.0), max_cycles=30)
    assert info.status != 0
    phi, rep = ndgp.solve(ndgp.Grid(n=n, h=h),
                          ndgp.Params(rc=rc, tol=1e-10, max_cycles=20, precision=prec),
                          [dev(d)], check=False)
    torch.cuda.synchronize()
    say(f"  status={rep.status} cycles={rep.cycles[0]} fallbacks={rep.fallbacks} "
        f"holds={rep.holds}")
    assert rep.status == ndgp.NDGP_ENOCONV
    assert rep.fallbacks > 0


# --------------------------------------------------------------------------
# the norms behind the force-difference report (Sec. III.B, Eqs. errors, errors2)

def test_diff_norms_against_numpy():
    """ndgp_diff_norms: sum (a-b)^2, sum a^2, sum b^2 in the library's fixed-order
    reduction, against exactly rounded sums (math.fsum), for counts that do not
    fill the reduction grid, with b = NULL, on a force-sized array, and the
    same bits on a second call."""
    import math
    rng = np.random.default_rng(5)
    for count in (1, 7, 1000, 4096 * 256 + 17, 3 * 64**3, 5_000_003):
        say(f"diff norms count={count}")
        a = rng.standard_normal(count) * 1e-3
        b = a + rng.standard_normal(count) * 1e-6
        ta, tb = dev(a), dev(b)
        d2, a2, b2 = ndgp.diff_norms(ta, tb)
        assert d2 == pytest.approx(math.fsum((a - b) ** 2), rel=1e-12)
        assert a2 == pytest.approx(math.fsum(a * a), rel=1e-12)
        assert b2 == pytest.approx(math.fsum(b * b), rel=1e-12)
        assert ndgp.diff_norms(ta, tb) == (d2, a2, b2)
        n2, m2, z2 = ndgp.diff_norms(ta)
        assert n2 == m2 == a2 and z2 == 0.0
    # the force report itself: interpolated vs relaxed patch force, 64^3 + patches
    f, deltas, grid = patch_problem()
    full, _ = gpu_solve(deltas, grid, rc=1.0, tol=1e-10, mode=ndgp.MODE_FULL)
    intp, _ = gpu_solve(deltas, grid, rc=1.0, tol=1e-10, mode=ndgp.MODE_INTERPOLATED)
    Ff = ndgp.force(grid, [dev(p) for p in full])
    Fi = ndgp.force(grid, [dev(p) for p in intp])
    for lvl in (1, 2):
        d2, i2, f2 = ndgp.diff_norms(Fi[lvl], Ff[lvl])
        fi, ff = Fi[lvl].cpu().numpy().ravel(), Ff[lvl].cpu().numpy().ravel()
        assert d2 == pytest.approx(math.fsum((fi - ff) ** 2), rel=1e-12)
        assert f2 == pytest.approx(math.fsum(ff * ff), rel=1e-12)
        say(f"  level {lvl}: |F_int - F_full| / |F_full| = {math.sqrt(d2 / f2):.3e}")
