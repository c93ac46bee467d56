"""Total force and effective gravity per refinement level.

TEST INFRASTRUCTURE ONLY: imported by the tests and never by the solver.
Plain float64 numpy, written from the definitions:

  Eq. (modpoisson)  the dynamical potential is Psi_N + phi/2, so the total
                    force is F = F_GR + F_5th with F_GR = -grad(Psi_N) and
                    F_5th = -grad(phi)/2 (central differences, Sec. III.B)
  Sec. III.B        G_eff = 1 + |F_5th| / |F_GR|
  Sec. IV.B, Fig. 3 G_eff against the finest refinement level: here every
                    cell counts on the finest level that holds it (a cell
                    covered by the next patch is left out of its own level)

Fields are the solver's layout: the periodic domain natural n^3, patches padded
(m+2)^3 with their ghost shells.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _padded(f, periodic):
    return O.pad_periodic(f) if periodic else np.ascontiguousarray(f, dtype=np.float64)


def total_force(phi, psi, h, periodic):
    """F_GR + F_5th, shape (3, n, n, n) (x, y, z): the oracle's central
    difference force of each potential, F_5th = force(phi) and
    F_GR = 2 force(psi) since force() returns -grad/2."""
    return 2.0 * O.force(psi, h, periodic) + O.force(phi, h, periodic)


def geff_minus_one(phi, psi, periodic):
    """|F_5th| / |F_GR| per cell, as sqrt(sum dphi^2 / sum dpsi^2) / 2 with the
    differences phi[c + e_a] - phi[c - e_a]; no Newtonian force: 0 without a
    fifth force, else inf."""
    p, s = _padded(phi, periodic), _padded(psi, periodic)
    n = p.shape[0] - 2
    c = slice(1, n + 1)
    up = [(c, c, slice(2, n + 2)), (c, slice(2, n + 2), c), (slice(2, n + 2), c, c)]
    dn = [(c, c, slice(0, n)), (c, slice(0, n), c), (slice(0, n), c, c)]
    a = np.zeros((n, n, n))
    b = np.zeros((n, n, n))
    for q in range(3):  # x, y, z, summed in that order
        dp = p[up[q]] - p[dn[q]]
        ds = s[up[q]] - s[dn[q]]
        a = a + dp * dp
        b = b + ds * ds
    with np.errstate(divide="ignore", invalid="ignore"):
        x = 0.5 * np.sqrt(a / b)
    x[(b == 0.0) & (a == 0.0)] = 0.0
    x[(b == 0.0) & (a != 0.0)] = np.inf
    return x


def uncovered(n, periodic, child_origin=None, child_n=0):
    """Boolean n^3 mask of the cells that the child box (child_n cells of half
    the size, lower corner child_origin in this level's cells) does not cover."""
    keep = np.ones((n, n, n), dtype=bool)
    if child_origin is None or child_n == 0:
        return keep
    half = child_n // 2
    idx = []
    for a in range(3):
        r = np.arange(child_origin[a], child_origin[a] + half)
        idx.append(r % n if periodic else r)
    keep[np.ix_(idx[2], idx[1], idx[0])] = False
    return keep


def geff_stats(phis, psis, origins, patch_ns, edges):
    """Per level: dict(cells, sum, sum_sq, min, max) of G_eff - 1 over the
    cells no finer patch covers, and the histogram over `edges` (bin 0: x <
    edges[0]; bin b: edges[b-1] <= x < edges[b]; last: x >= edges[-1])."""
    out, hists = [], []
    nl = len(phis)
    for l in range(nl):
        periodic = l == 0
        x = geff_minus_one(phis[l], psis[l], periodic)
        n = x.shape[0]
        keep = uncovered(n, periodic, origins[l] if l < nl - 1 else None,
                         patch_ns[l] if l < nl - 1 else 0)
        v = x[keep]
        out.append({"cells": int(v.size), "sum": float(np.sum(v)),
                    "sum_sq": float(np.sum(v * v)), "min": float(v.min()),
                    "max": float(v.max())})
        hists.append(np.bincount(np.searchsorted(np.asarray(edges), v, side="right"),
                                 minlength=len(edges) + 1))
    return out, np.array(hists, dtype=np.int64)
