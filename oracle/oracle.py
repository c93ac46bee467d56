"""Python face of the CPU oracle (``ndgp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package's smoke check and
the benchmark's CPU-baseline leg, never by the solver itself.  It does not
import the solver package and the solver does not import it.

Every function works in physical units (lengths in c/H0, phi in c^2) on float64
arrays in natural layout ``[z][y][x]`` unless it says "padded" (``(n+2)^3``
with a one-cell ghost shell).  The arithmetic lives in the C file; here there is
only marshalling and the top-level order of the paper's algorithm
(Sec. III.A: periodic domain level first, then each refinement level from its
parent; Sec. III.B: refinements optionally left at their interpolated guess).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import dataclasses

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ndgp_oracle.c")
_LIB = os.path.join(_HERE, "libndgp_oracle.so")

C_OVER_H0_MPC_H = 2997.92458  # c/H0 in Mpc/h


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64 = ctypes.c_int64
        L.oracle_beta_lcdm.restype = ctypes.c_double
        L.oracle_beta_lcdm.argtypes = [ctypes.c_double] * 3
        L.oracle_alpha.restype = ctypes.c_double
        L.oracle_alpha.argtypes = [ctypes.c_double] * 3
        L.oracle_source.argtypes = [i64, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    dp, dp]
        L.oracle_source_shift.argtypes = [i64, dp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, dp]
        L.oracle_operator.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, dp, dp]
        L.oracle_operator_at.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp,
                                         i64, ctypes.POINTER(ctypes.c_int32), dp]
        L.oracle_newton_update.restype = ctypes.c_double
        L.oracle_newton_update.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]
        L.oracle_interpolate.restype = ctypes.c_int
        L.oracle_interpolate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
                                         ctypes.c_int, dp, ctypes.c_int]
        L.oracle_solve_periodic.restype = ctypes.c_int
        L.oracle_solve_periodic.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp,
                                            dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, dp]
        L.oracle_solve_patch.restype = ctypes.c_int
        u8p = ctypes.POINTER(ctypes.c_ubyte)
        L.oracle_solve_patch.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp,
                                         ctypes.c_int, ctypes.c_int, ip, dp, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, u8p, dp, ctypes.c_int, ip, dp]
        L.oracle_cell_mask.restype = ctypes.c_int
        L.oracle_cell_mask.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
                                       ctypes.c_double, u8p]
        L.oracle_force.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# --------------------------------------------------------------------------
# background, Sec. II

def beta_lcdm(a: float, omega_m: float, rc: float) -> float:
    """beta(a) of Eq. (beta) on the LCDM expansion history (r_c in c/H0)."""
    return float(lib().oracle_beta_lcdm(a, omega_m, rc))


def alpha(rc: float, beta: float, a: float) -> float:
    """r_c^2 / (3 beta a^2), the coefficient of Eq. (eomvarphi)'s nonlinear term."""
    return float(lib().oracle_alpha(rc, beta, a))


def cell_size(box_mpc_h: float, n: int) -> float:
    """Cell size in c/H0 of an n^3 grid over a box of side box_mpc_h (Mpc/h)."""
    return box_mpc_h / n / C_OVER_H0_MPC_H


def source(delta, omega_m: float, a: float, beta: float):
    """S = Omega_m (delta - mean delta) / (a beta); returns (S, removed mean)."""
    d = _c(delta)
    S = np.empty_like(d)
    m = ctypes.c_double()
    lib().oracle_source(d.size, _dp(d), omega_m, a, beta, _dp(S), ctypes.byref(m))
    return S, m.value


def source_shift(delta, mean: float, omega_m: float, a: float, beta: float):
    d = _c(delta)
    S = np.empty_like(d)
    lib().oracle_source_shift(d.size, _dp(d), mean, omega_m, a, beta, _dp(S))
    return S


# --------------------------------------------------------------------------
# operator

def pad_periodic(phi) -> np.ndarray:
    return np.pad(_c(phi), 1, mode="wrap")


def operator(phi, h: float, alpha_: float) -> np.ndarray:
    """L_h[phi] on a periodic natural-layout field."""
    p = pad_periodic(phi)
    n = phi.shape[0]
    out = np.empty((n, n, n))
    lib().oracle_operator(n, 1, h, alpha_, _dp(p), _dp(out))
    return out


def operator_padded(phi_pad, h: float, alpha_: float) -> np.ndarray:
    """L_h[phi] on the interior of a padded field whose ghosts are given."""
    p = _c(phi_pad).copy()
    n = p.shape[0] - 2
    out = np.empty((n, n, n))
    lib().oracle_operator(n, 0, h, alpha_, _dp(p), _dp(out))
    return out


def operator_at(phi, h: float, alpha_: float, cells) -> np.ndarray:
    """L_h[phi] at the listed (i, j, k) cells of a periodic natural field."""
    ph = _c(phi)
    c = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
    out = np.empty(len(c))
    lib().oracle_operator_at(ph.shape[0], h, alpha_, _dp(ph), len(c),
                             c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(out))
    return out


def newton_update(phi_pad, h: float, alpha_: float, S_cell: float, i: int, j: int, k: int) -> float:
    """One Newton step of Eq. (newton) at cell (i, j, k) of a padded field."""
    p = _c(phi_pad)
    return float(lib().oracle_newton_update(p.shape[0] - 2, h, alpha_, _dp(p), S_cell, i, j, k))


def interpolate(parent, parent_periodic: bool, origin, m: int, nc: int,
                child_pad=None, ghosts_only: bool = False) -> np.ndarray:
    """Trilinear, cell-centred interpolation of a parent level onto a child box
    (lower corner ``origin`` = (x, y, z) in parent cells, child cell = 2^m / 2
    parent cells).  Returns the padded child."""
    par = _c(parent)
    np_ = par.shape[0] if parent_periodic else par.shape[0] - 2
    out = np.zeros((nc + 2,) * 3) if child_pad is None else _c(child_pad).copy()
    o = (ctypes.c_int * 3)(*[int(v) for v in origin])
    rc = lib().oracle_interpolate(_dp(par), np_, 1 if parent_periodic else 0, o, m, nc,
                                  _dp(out), 1 if ghosts_only else 0)
    if rc:
        raise ValueError("child box reaches outside the parent")
    return out


# --------------------------------------------------------------------------
# solves

@dataclasses.dataclass
class SolveInfo:
    status: int
    cycles: int
    rel_res: float
    history: np.ndarray


def solve_periodic(S, h: float, alpha_: float, phi0=None, max_cycles: int = 200,
                   tol: float = 0.0, nu1: int = 2, nu2: int = 2):
    """Periodic domain solve; tol <= 0 runs to stagnation.  ``phi0`` is a warm
    start; without it the initial guess comes from nested iteration.  Returns
    (phi, info), phi with zero mean."""
    Sc = _c(S)
    n = Sc.shape[0]
    phi = np.zeros_like(Sc) if phi0 is None else _c(phi0).copy()
    hist = np.zeros(max(max_cycles, 1))
    cyc = ctypes.c_int()
    rel = ctypes.c_double()
    st = lib().oracle_solve_periodic(n, h, alpha_, _dp(Sc), _dp(phi), 0 if phi0 is None else 1,
                                     max_cycles, tol, nu1, nu2,
                                     _dp(hist), len(hist), ctypes.byref(cyc), ctypes.byref(rel))
    return phi, SolveInfo(st, cyc.value, rel.value, hist[:cyc.value].copy())


def solve_patch(S, h: float, alpha_: float, parent, parent_periodic: bool, origin,
                interp_only: bool = False, max_cycles: int = 200, tol: float = 0.0,
                nu1: int = 2, nu2: int = 2, mask=None):
    """Refined-patch solve with boundary values and initial guess interpolated
    from the parent (periodic natural or padded).  ``mask`` (uint8, natural
    nc^3): cells with 0 keep the interpolated guess and are not part of the
    equations solved (cell-wise truncation).  Returns (phi_pad, info)."""
    Sc = _c(S)
    nc = Sc.shape[0]
    par = _c(parent)
    np_ = par.shape[0] if parent_periodic else par.shape[0] - 2
    out = np.zeros((nc + 2,) * 3)
    o = (ctypes.c_int * 3)(*[int(v) for v in origin])
    hist = np.zeros(max(max_cycles, 1))
    cyc = ctypes.c_int()
    rel = ctypes.c_double()
    mk = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mk.shape == (nc, nc, nc)
    st = lib().oracle_solve_patch(nc, h, alpha_, _dp(Sc), _dp(par), np_,
                                  1 if parent_periodic else 0, o, _dp(out), max_cycles, tol,
                                  nu1, nu2, 1 if interp_only else 0,
                                  None if mk is None else mk.ctypes.data_as(
                                      ctypes.POINTER(ctypes.c_ubyte)),
                                  _dp(hist), len(hist), ctypes.byref(cyc), ctypes.byref(rel))
    if st == -1:
        raise ValueError("patch reaches outside its parent")
    return out, SolveInfo(st, cyc.value, rel.value, hist[:cyc.value].copy())


def cell_mask(phi_parent, psi_parent, parent_periodic: bool, origin, nc: int,
              threshold: float) -> np.ndarray:
    """Sec. III.C: 1 where the parent cell's fifth force is at least
    ``threshold`` times its Newtonian force (central differences of phi/2 and
    of the Newtonian potential psi on the parent level), else 0.  Parents are
    periodic natural or padded; returns uint8 natural nc^3."""
    ph, ps = _c(phi_parent), _c(psi_parent)
    assert ph.shape == ps.shape
    np_ = ph.shape[0] if parent_periodic else ph.shape[0] - 2
    out = np.zeros((nc, nc, nc), dtype=np.uint8)
    o = (ctypes.c_int * 3)(*[int(v) for v in origin])
    rc = lib().oracle_cell_mask(_dp(ph), _dp(ps), np_, 1 if parent_periodic else 0, o, nc,
                                float(threshold), out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    if rc:
        raise ValueError("child box reaches outside the parent")
    return out


def force(phi, h: float, periodic: bool = True) -> np.ndarray:
    """F = -grad(phi)/2, central differences; (3, n, n, n) with x, y, z."""
    p = pad_periodic(phi) if periodic else _c(phi).copy()
    n = p.shape[0] - 2
    f = np.empty((3, n, n, n))
    lib().oracle_force(n, h, _dp(p), 1 if periodic else 0, _dp(f))
    return f


@dataclasses.dataclass
class Problem:
    """Everything one solve needs, in the paper's parameters."""
    delta: list            # [base (n^3), patch1, patch2] natural float64
    h: float               # base cell size, c/H0
    rc: float              # r_c H0
    beta: float
    a: float = 1.0
    omega_m: float = 0.3
    origins: tuple = ()    # per patch, lower corner (x, y, z) in parent cells


def solve_problem(p: Problem, interpolated: bool = False, tol: float = 0.0,
                  max_cycles: int = 200, trunc_level: int | None = None, cellwise=None):
    """The whole path: domain level, then every patch level from its parent
    (Sec. III.A), or by interpolation only (Sec. III.B).  ``trunc_level`` k
    relaxes patch levels 1..k-1 and interpolates levels k and up, each from
    its own (relaxed or interpolated) parent: the truncation l >= l_trunc of
    Sec. IV.A with l_trunc = l_d + k.  k = 1 is ``interpolated=True``.
    ``cellwise = (psi, threshold)``: on every relaxed patch only the cells whose
    parent cell has |F_5th| >= threshold |F_GR| are iterated (Sec. III.C), with
    psi[l] the Newtonian potential of level l (natural domain, padded patches).
    Returns (phis, infos, masks) with cellwise, else (phis, infos): phis[0]
    natural zero-mean, phis[1:] padded with ghosts."""
    if trunc_level is None:
        trunc_level = 1 if interpolated else len(p.delta)
    al = alpha(p.rc, p.beta, p.a)
    S0, mean = source(p.delta[0], p.omega_m, p.a, p.beta)
    phi0, info0 = solve_periodic(S0, p.h, al, tol=tol, max_cycles=max_cycles)
    phis, infos = [phi0], [info0]
    parent, parent_periodic, h = phi0, True, p.h
    masks = [None]
    for lvl in range(1, len(p.delta)):
        h = h / 2
        S = source_shift(p.delta[lvl], mean, p.omega_m, p.a, p.beta)
        mk = None
        if cellwise is not None and lvl < trunc_level:
            psi, thr = cellwise
            mk = cell_mask(parent, psi[lvl - 1], parent_periodic, p.origins[lvl - 1],
                           S.shape[0], thr)
        ph, inf = solve_patch(S, h, al, parent, parent_periodic, p.origins[lvl - 1],
                              interp_only=lvl >= trunc_level, tol=tol, max_cycles=max_cycles,
                              mask=mk)
        phis.append(ph)
        infos.append(inf)
        masks.append(mk)
        parent, parent_periodic = ph, False
    if cellwise is not None:
        return phis, infos, masks
    return phis, infos


def solve_tree(delta, h: float, rc: float, beta: float, boxes, a: float = 1.0,
               omega_m: float = 0.3, interpolated: bool = False, trunc_depth=None,
               tol: float = 0.0, max_cycles: int = 200):
    """Sec. III.A's order on a tree of refinements (several per level, Sec.
    IV.A): the periodic domain, then every box from its own parent, in list
    order.  ``boxes``: (parent, n, origin) per box, parent -1 for the domain,
    origin in parent cells; ``delta``: [domain, box 0, ...].  A box of tree
    depth d has cells h / 2^d.  Boxes are interpolated (Sec. III.B) when
    ``interpolated`` or their depth is at least ``trunc_depth``.  Returns
    (phis, infos): phis[0] natural zero-mean, phis[1:] padded."""
    al = alpha(rc, beta, a)
    S0, mean = source(delta[0], omega_m, a, beta)
    phi0, info0 = solve_periodic(S0, h, al, tol=tol, max_cycles=max_cycles)
    phis, infos, depth = [phi0], [info0], []
    for b, (parent, n, origin) in enumerate(boxes):
        d = 1 if parent < 0 else depth[parent] + 1
        depth.append(d)
        interp = interpolated or (trunc_depth is not None and d >= trunc_depth)
        S = (np.zeros((n, n, n)) if interp
             else source_shift(delta[1 + b], mean, omega_m, a, beta))
        par = phis[0] if parent < 0 else phis[1 + parent]
        ph, inf = solve_patch(S, h / 2**d, al, par, parent < 0, origin, interp_only=interp,
                              tol=tol, max_cycles=max_cycles)
        phis.append(ph)
        infos.append(inf)
    return phis, infos
