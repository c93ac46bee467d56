"""Seeded synthetic density fields: the one module shared by the solver's tests,
the benchmark and the CPU oracle's tests.

It only draws random numbers and shapes them into a density contrast
``delta = rho / mean(rho) - 1``; it knows nothing of the scalar-field equation.

The paper's solver runs on cloud-in-cell densities of an N-body simulation
(Sec. IV.A: L = 250 Mpc/h, 512^3 particles).  No particles or snapshots exist
here, so a lognormal field with a power-law spectrum plus spherical top-hat
overdensities stands in for them: the lognormal gives the long high-density
tail of a nonlinear matter field, the top-hats give isolated screened objects
like the ones of Sec. II.A (Eqs. eomvarphi_sph - forcesmall).

Layout: every array is float64, shape (n, n, n), index order [z][y][x] with x
fastest (C order).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "TopHat",
    "Field",
    "lognormal_rho",
    "draw_tophats",
    "paint_tophats",
    "make_field",
    "patch_delta",
    "densest_tophat_centre",
    "patch_origin_centred",
    "lognormal_delta_torch",
    "make_particles",
]


@dataclasses.dataclass(frozen=True)
class TopHat:
    """A spherical overdensity: centre in units of base cells (continuous,
    cell c spans [c, c+1)), radius in base cells, and added density in units
    of the lognormal mean."""
    cx: float
    cy: float
    cz: float
    radius: float
    amplitude: float


@dataclasses.dataclass
class Field:
    """A base-grid density contrast and what it was built from."""
    delta: np.ndarray          # (n, n, n) float64, zero mean up to rounding
    rho_lognormal: np.ndarray  # (n, n, n) the lognormal part, mean 1
    tophats: list
    rho_mean: float            # mean of lognormal + top-hats (normaliser of delta)


def lognormal_rho(n: int, sigma: float, seed: int, slope: float = -2.0) -> np.ndarray:
    """Lognormal density with mean 1.

    A white Gaussian field is filtered in Fourier space by |k|^(slope/2)
    (power spectrum P(k) ~ k^slope) inside the sphere |k| <= k_Nyquist, with
    the k = 0 mode removed.  The result is standardised to variance sigma^2
    (sample statistics), exponentiated and divided by its mean.
    """
    if n < 2 or n & (n - 1):
        raise ValueError("n must be a power of two >= 2")
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    del w
    kz = np.fft.fftfreq(n) * n
    ky = np.fft.fftfreq(n) * n
    kx = np.fft.rfftfreq(n) * n
    k2 = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2) + kx[None, None, :] ** 2
    kmax2 = (n / 2) ** 2
    with np.errstate(divide="ignore"):
        filt = np.where((k2 > 0) & (k2 <= kmax2), k2 ** (slope / 4.0), 0.0)
    wk *= filt
    del filt, k2
    g = np.fft.irfftn(wk, s=(n, n, n), axes=(0, 1, 2))
    del wk
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g *= sigma / sd
    np.exp(g, out=g)
    g /= g.mean()
    return g


def draw_tophats(n: int, count: int, seed: int, rmin: float = 2.0, rmax: float = 8.0,
                 amplitude: float = 200.0) -> list:
    """``count`` top-hats with centres uniform in the box and radii uniform in
    [rmin, rmax] base cells."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, float(n), size=(count, 3))
    r = rng.uniform(rmin, rmax, size=count)
    return [TopHat(float(c[i, 0]), float(c[i, 1]), float(c[i, 2]), float(r[i]), amplitude)
            for i in range(count)]


def _periodic_sep(coord: np.ndarray, centre: float, period: float) -> np.ndarray:
    d = coord - centre
    return d - period * np.round(d / period)


def paint_tophats(rho: np.ndarray, tophats: list, n_base: int, origin=(0.0, 0.0, 0.0),
                  cell: float = 1.0) -> None:
    """Add every top-hat to ``rho`` in place, testing the distance of each cell
    centre (periodic in the base box) against the radius; overlaps add.

    ``rho`` covers a box whose lower corner is ``origin`` (base-cell units, per
    axis x, y, z) with cells of size ``cell`` base cells.
    """
    nz, ny, nx = rho.shape
    xs = origin[0] + (np.arange(nx) + 0.5) * cell
    ys = origin[1] + (np.arange(ny) + 0.5) * cell
    zs = origin[2] + (np.arange(nz) + 0.5) * cell
    for t in tophats:
        dx = _periodic_sep(xs, t.cx, n_base)
        dy = _periodic_sep(ys, t.cy, n_base)
        dz = _periodic_sep(zs, t.cz, n_base)
        ix = np.nonzero(np.abs(dx) <= t.radius)[0]
        iy = np.nonzero(np.abs(dy) <= t.radius)[0]
        iz = np.nonzero(np.abs(dz) <= t.radius)[0]
        if not (len(ix) and len(iy) and len(iz)):
            continue
        d2 = (dz[iz][:, None, None] ** 2 + dy[iy][None, :, None] ** 2) + dx[ix][None, None, :] ** 2
        inside = d2 <= t.radius ** 2
        sub = rho[np.ix_(iz, iy, ix)]
        sub += inside * t.amplitude
        rho[np.ix_(iz, iy, ix)] = sub


def make_field(n: int, sigma: float, seed: int, n_tophats: int = 0,
               tophat_amplitude: float = 200.0) -> Field:
    """Base-grid field: lognormal (seed) plus ``n_tophats`` top-hats (seed + 1),
    normalised so that ``delta = rho/mean(rho) - 1``."""
    rho_ln = lognormal_rho(n, sigma, seed)
    rho = rho_ln.copy()
    ths = draw_tophats(n, n_tophats, seed + 1, amplitude=tophat_amplitude) if n_tophats else []
    if ths:
        paint_tophats(rho, ths, n)
    m = float(rho.mean())
    delta = rho / m
    delta -= 1.0
    return Field(delta=delta, rho_lognormal=rho_ln, tophats=ths, rho_mean=m)


def densest_tophat_centre(field: Field):
    """Centre (base-cell units, x, y, z) of the largest-radius top-hat (lowest
    index on ties); without top-hats, the centre of the densest cell."""
    if field.tophats:
        best = max(range(len(field.tophats)), key=lambda i: (field.tophats[i].radius, -i))
        t = field.tophats[best]
        return (t.cx, t.cy, t.cz)
    k, j, i = np.unravel_index(int(np.argmax(field.delta)), field.delta.shape)
    return (i + 0.5, j + 0.5, k + 0.5)


def patch_origin_centred(centre_parent_units, cover_parent_cells: int):
    """Integer lower corner (x, y, z, parent-cell units) of a cube of
    ``cover_parent_cells`` parent cells centred on ``centre_parent_units``."""
    return tuple(int(math.floor(c - cover_parent_cells / 2.0 + 0.5)) for c in centre_parent_units)


def patch_delta(field: Field, n_base: int, chain, n_patch: int) -> np.ndarray:
    """Density contrast on a refined patch.

    ``chain`` lists, from the base level down to this patch, the integer lower
    corners (x, y, z) of every patch in its parent's cell units; each level
    halves the cell size.  The lognormal part is injected piecewise constant
    from the base cell that contains each patch cell centre, the top-hats are
    evaluated at the patch cell centres, and the sum is normalised by the base
    mean density, so the patch sees the same objects at finer resolution.
    """
    # lower corner of the patch and its cell size, in base-cell units
    corner = np.zeros(3)
    cell = 1.0
    for o in chain:
        corner = corner + np.asarray(o, dtype=np.float64) * cell
        cell *= 0.5
    centres = [corner[a] + (np.arange(n_patch) + 0.5) * cell for a in range(3)]
    base_idx = [np.floor(c).astype(np.int64) % n_base for c in centres]
    rho = field.rho_lognormal[np.ix_(base_idx[2], base_idx[1], base_idx[0])].copy()
    if field.tophats:
        paint_tophats(rho, field.tophats, n_base, origin=tuple(corner), cell=cell)
    rho /= field.rho_mean
    rho -= 1.0
    return rho


def lognormal_delta_torch(n: int, sigma: float, seed: int, device="cuda", slope: float = -2.0):
    """The lognormal recipe of ``lognormal_rho`` drawn with torch on a device
    (for request streams, where host generation would dominate), returned as
    the density contrast rho / mean(rho) - 1.  Deterministic for a given seed
    and device; not the same numbers as the numpy generator."""
    import torch
    if n < 2 or n & (n - 1):
        raise ValueError("n must be a power of two >= 2")
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    w = torch.randn((n, n, n), generator=g, device=device, dtype=torch.float64)
    wk = torch.fft.rfftn(w)
    del w
    kz = torch.fft.fftfreq(n, device=device, dtype=torch.float64) * n
    kx = torch.fft.rfftfreq(n, device=device, dtype=torch.float64) * n
    k2 = (kz[:, None, None] ** 2 + kz[None, :, None] ** 2) + kx[None, None, :] ** 2
    keep = (k2 > 0) & (k2 <= (n / 2) ** 2)
    filt = torch.where(keep, k2.clamp_min(1e-300) ** (slope / 4.0), torch.zeros_like(k2))
    wk *= filt
    del filt, k2, keep
    f = torch.fft.irfftn(wk, s=(n, n, n))
    del wk
    f -= f.mean()
    sd = f.std(unbiased=False)
    f *= sigma / sd
    torch.exp(f, out=f)
    f /= f.mean()
    f -= 1.0
    return f.contiguous()


def make_particles(field: Field, n_particles: int, seed: int,
                   cell_order: bool = False) -> np.ndarray:
    """Equal-mass particles that sample a field: each particle picks a base
    cell with probability proportional to rho = 1 + delta there, then a
    uniform position inside it.  Returns float64 (3, n_particles): x, y, z in
    units of the box, each in [0, 1) (structure of arrays).  The particles
    come in random order, or sorted by base cell with cell_order (the order
    a tree code keeps them in)."""
    n = field.delta.shape[0]
    rng = np.random.default_rng(seed)
    p = np.maximum(field.delta.ravel() + 1.0, 0.0)
    p = p / p.sum()
    counts = rng.multinomial(n_particles, p)
    cells = np.repeat(np.arange(p.size), counts)
    perm = rng.permutation(n_particles)
    if not cell_order:
        cells = cells[perm]  # particles in no spatial order
    k, j, i = np.unravel_index(cells, (n, n, n))
    u = rng.random((3, n_particles))
    pos = np.empty((3, n_particles))
    pos[0] = (i + u[0]) / n
    pos[1] = (j + u[1]) / n
    pos[2] = (k + u[2]) / n
    np.minimum(pos, np.nextafter(1.0, 0.0), out=pos)  # stay inside [0, 1)
    return pos
