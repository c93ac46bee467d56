"""Cloud-in-cell transfers between particles and the grid levels (Sec. IV.A:
the density and the forces are interpolated back and forth between the
particles and the AMR cells by cloud-in-cell).

TEST INFRASTRUCTURE ONLY: imported by the tests and never by the solver.
Plain float64 numpy written from the definition of cloud-in-cell: a particle
is a cube of one cell's size centred on its position; it gives each cell the
overlapping fraction of its mass, which for cell-centred grids is the product
over the three axes of (1 - t) for the cell whose centre lies below the
particle and t for the next one, t being the distance from the lower centre in
cells.  Force interpolation uses the same weights.

Geometry follows the solver: level 0 is the periodic domain (n^3 cells), level
q >= 1 a patch of m^3 cells of size 2^-q domain cells whose lower corner, in
domain cells, is the sum of the chain of integer origins (each in its
parent's cells).  Positions are in units of the box, in [0, 1).  Patches may
wrap the periodic domain, so positions are compared with a patch modulo the
box (both images of a particle near the box edge are tried).
"""
from __future__ import annotations

import numpy as np


def level_corners(origins):
    """Lower corner (x, y, z) of every level in domain cells: level 0 at 0,
    level q at corner(q-1) + origin(q-1) 2^-(q-1)."""
    corners = [np.zeros(3)]
    for q, o in enumerate(origins):
        corners.append(corners[-1] + np.asarray(o, dtype=np.float64) * 2.0 ** (-q))
    return corners


def _axis_terms(x_cells, corner, q, m, periodic, n):
    """Per particle, the (cell index, weight) pairs along one axis that fall
    inside [0, m): lists of arrays (index, weight, valid)."""
    d = x_cells - corner
    d = d - n * np.floor(d / n)              # in [0, n)
    out = []
    images = (d,) if periodic else (d, d - n)
    for img in images:
        u = img * 2.0**q - 0.5               # in cells of this level, centres at integers
        i0 = np.floor(u)
        t = u - i0
        for off, w in ((0, 1.0 - t), (1, t)):
            idx = i0.astype(np.int64) + off
            if periodic:
                out.append((idx % m, w, np.ones_like(w, dtype=bool)))
            else:
                out.append((idx, w, (idx >= 0) & (idx < m)))
    return out


def deposit(pos, n, origins=(), patch_ns=()):
    """Cloud-in-cell density contrast on every level: delta = count / mean -
    1 with mean = N / (n 2^q)^3 particles per level-q cell (the domain's mean
    density, as the solver's patch densities are measured)."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[1]
    corners = level_corners(origins)
    sizes = [n] + list(patch_ns)
    deltas = []
    for q, m in enumerate(sizes):
        periodic = q == 0
        terms = [_axis_terms(pos[a] * n, corners[q][a], q, m, periodic, n) for a in range(3)]
        count = np.zeros(m * m * m)
        for iz, wz, vz in terms[2]:
            for iy, wy, vy in terms[1]:
                for ix, wx, vx in terms[0]:
                    ok = vx & vy & vz
                    flat = (iz[ok] * m + iy[ok]) * m + ix[ok]
                    np.add.at(count, flat, (wx * wy * wz)[ok])
        mean = N / float(n * 2**q) ** 3
        deltas.append((count / mean - 1.0).reshape(m, m, m))
    return deltas


def gather(forces, pos, n, origins=(), patch_ns=()):
    """Cloud-in-cell interpolation of per-level fields (3, m, m, m) to the
    particles, each from the finest level whose eight cells around it all lie
    inside that level (the domain always qualifies).  Returns (3, N)."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[1]
    corners = level_corners(origins)
    sizes = [n] + list(patch_ns)
    out = np.zeros((3, N))
    done = np.zeros(N, dtype=bool)
    for q in range(len(sizes) - 1, -1, -1):
        m = sizes[q]
        periodic = q == 0
        lo, wt = [], []
        ok = ~done
        for a in range(3):
            d = pos[a] * n - corners[q][a]
            d = d - n * np.floor(d / n)
            best_i = np.full(N, -10**9, dtype=np.int64)
            best_t = np.zeros(N)
            for img in ((d,) if periodic else (d, d - n)):
                u = img * 2.0**q - 0.5
                i0 = np.floor(u)
                inside = periodic | ((i0 >= 0) & (i0 + 1 <= m - 1))
                best_i = np.where(inside, i0.astype(np.int64), best_i)
                best_t = np.where(inside, u - i0, best_t)
            ok &= periodic | (best_i >= 0)
            lo.append(best_i)
            wt.append(best_t)
        idx = np.nonzero(ok)[0]
        f = forces[q].reshape(3, -1)
        acc = np.zeros((3, idx.size))
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = ((wt[0][idx] if dx else 1 - wt[0][idx]) * (wt[1][idx] if dy else 1 - wt[1][idx])
                         * (wt[2][idx] if dz else 1 - wt[2][idx]))
                    cx, cy, cz = lo[0][idx] + dx, lo[1][idx] + dy, lo[2][idx] + dz
                    if periodic:
                        cx, cy, cz = cx % m, cy % m, cz % m
                    acc += w * f[:, (cz * m + cy) * m + cx]
        out[:, idx] = acc
        done[idx] = True
    return out


def deposit_at(pos, n, cells, chunk=1 << 21):
    """Domain-level cloud-in-cell density contrast at selected cells only
    (flat indices (k n + j) n + i), the same definition as deposit(), for
    particle sets too large to deposit whole.  Works through the particles in
    chunks."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[1]
    cells = np.asarray(cells, dtype=np.int64)
    order = np.argsort(cells)
    sorted_cells = cells[order]
    count = np.zeros(cells.size)
    for s in range(0, N, chunk):
        p = pos[:, s:s + chunk]
        terms = [_axis_terms(p[a] * n, 0.0, 0, n, True, n) for a in range(3)]
        for iz, wz, _ in terms[2]:
            for iy, wy, _ in terms[1]:
                for ix, wx, _ in terms[0]:
                    flat = (iz * n + iy) * n + ix
                    at = np.searchsorted(sorted_cells, flat)
                    at = np.minimum(at, sorted_cells.size - 1)
                    hit = sorted_cells[at] == flat
                    np.add.at(count, order[at[hit]], (wx * wy * wz)[hit])
    return count / (N / float(n) ** 3) - 1.0
