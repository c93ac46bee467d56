"""Pins of the cloud-in-cell oracle (oracle/cic.py; Sec. IV.A: density and
forces move between particles and cells by cloud-in-cell) against facts that
do not come from it: mass conservation, the weights at cell centres and
corners, a uniform lattice, exactness on linear fields, and gather being the
transpose of deposit.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import cic as C
from paper_1511_08200_amd import synth


def test_mass_conservation_and_mean():
    rng = np.random.default_rng(1)
    pos = rng.random((3, 5000))
    (d,) = C.deposit(pos, 16)
    assert d.mean() == pytest.approx(0.0, abs=1e-13)       # sum of counts = N
    assert (d >= -1.0).all()


def test_weights_at_centres_and_corners():
    n = 8
    # at the centre of cell (2, 5, 7): all of the mass there
    pos = np.array([[2.5 / n], [5.5 / n], [7.5 / n]])
    (d,) = C.deposit(pos, n)
    count = (d + 1.0) / n**3
    assert count[7, 5, 2] == pytest.approx(1.0, abs=1e-14)
    assert np.count_nonzero(np.abs(count) > 1e-14) == 1
    # at the shared corner of cells (0..1)^3, wrapping: x = 0 sits between 7 and 0
    pos = np.array([[0.0], [1.0 / n], [1.0 / n]])
    (d,) = C.deposit(pos, n)
    count = (d + 1.0) / n**3
    for (k, j, i) in [(0, 0, 7), (0, 0, 0), (1, 1, 7), (1, 1, 0), (0, 1, 0), (1, 0, 7)]:
        assert count[k, j, i] == pytest.approx(0.125, abs=1e-14)


def test_uniform_lattice_is_uniform():
    n = 8
    g = (np.arange(2 * n) + 0.5) / (2 * n)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    (d,) = C.deposit(pos, n)
    np.testing.assert_allclose(d, 0.0, atol=1e-12)


def test_patch_levels_and_wrapping():
    """A patch (m cells of half size) that wraps the box edge receives the same
    counts as the domain refined by two, from particles on both sides of the
    edge."""
    rng = np.random.default_rng(3)
    n, m = 16, 16
    pos = rng.random((3, 20000))
    origin = (-4, 3, 5)        # patch 1 covers domain cells -4..3 in x (wraps)
    d0, d1 = C.deposit(pos, n, origins=[origin], patch_ns=[m])
    # the same particles deposited on a 32^3 domain: the patch is a window of it
    (dd,) = C.deposit(pos, 2 * n)
    win = dd[np.ix_((2 * origin[2] + np.arange(m)) % 32, (2 * origin[1] + np.arange(m)) % 32,
                    (2 * origin[0] + np.arange(m)) % 32)]
    np.testing.assert_allclose(d1, win, atol=1e-11)


def test_gather_exact_on_linear_fields_and_transpose():
    rng = np.random.default_rng(4)
    n, m = 16, 16
    origin = (4, 4, 4)
    # particles well inside the patch: its linear force field is reproduced
    pos = (np.array(origin)[:, None] + 1.0 + 6.0 * rng.random((3, 300))) / n
    zc = (np.arange(m) + 0.5) / 2 + origin[2]
    yc = (np.arange(m) + 0.5) / 2 + origin[1]
    xc = (np.arange(m) + 0.5) / 2 + origin[0]
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    lin = np.stack([2 * X - Y, Z + 0.5, -3 * X + Y + Z])
    F0 = np.zeros((3, n, n, n))
    out = C.gather([F0, lin], pos, n, origins=[origin], patch_ns=[m])
    P = pos * n
    want = np.stack([2 * P[0] - P[1], P[2] + 0.5, -3 * P[0] + P[1] + P[2]])
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-12)
    # on the domain alone, gather is the transpose of deposit:
    # sum_p F(x_p) = sum_cells count * F
    pos = rng.random((3, 4000))
    F = rng.standard_normal((3, n, n, n))
    (d,) = C.deposit(pos, n)
    count = (d + 1.0) * pos.shape[1] / n**3
    g = C.gather([F], pos, n)
    for a in range(3):
        assert g[a].sum() == pytest.approx((count * F[a]).sum(), rel=1e-11)


def test_particle_sampler_follows_the_field():
    f = synth.make_field(16, 1.5, 5, n_tophats=2)
    pos = synth.make_particles(f, 400000, 9)
    assert pos.shape == (3, 400000) and pos.min() >= 0.0 and pos.max() < 1.0
    idx = np.floor(pos * 16).astype(int)
    counts = np.bincount((idx[2] * 16 + idx[1]) * 16 + idx[0], minlength=16**3)
    expect = (f.delta.ravel() + 1.0) / (f.delta.ravel() + 1.0).sum() * 400000
    assert np.corrcoef(counts, expect)[0, 1] > 0.99


def test_deposit_at_selected_cells_is_deposit():
    rng = np.random.default_rng(8)
    pos = rng.random((3, 30000))
    (d,) = C.deposit(pos, 16)
    cells = rng.choice(16**3, size=200, replace=False)
    np.testing.assert_allclose(C.deposit_at(pos, 16, cells, chunk=7000), d.ravel()[cells],
                               rtol=0, atol=1e-12)
