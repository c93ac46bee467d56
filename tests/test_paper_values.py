"""Consistency of the numbers the paper prints (tests/golden/paper_values.json)
with the unit conventions used by the oracle and the library."""
from __future__ import annotations

import json
import math
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")
RHO_CRIT_H2 = 2.77536627e11  # critical density today, h^2 Msun / Mpc^3 (3 H0^2 / 8 pi G)


@pytest.fixture(scope="module")
def pv():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_domain_level_and_cell_sizes(pv, oracle_mod):
    sim = pv["simulation"]
    L, npart = sim["box_mpc_h"], sim["particles_per_side"]
    assert 2 ** sim["domain_level"] == npart  # 2^l_d = N_p^(1/3)

    def truncated(x, digits=2):  # the paper prints cell sizes cut to two decimals
        return math.floor(x * 10**digits) / 10**digits

    assert truncated(L / 2 ** sim["domain_level"]) == sim["domain_cell_mpc_h"]
    for lvl, hc in pv["truncation"]["levels"].items():
        assert truncated(L / 2 ** int(lvl)) == hc
    # the oracle's cell size in c/H0 converts back to the printed Mpc/h value
    h = oracle_mod.cell_size(L, 2 ** sim["domain_level"])
    assert h * 2997.92458 == pytest.approx(L / 512, rel=1e-15)


def test_particle_mass(pv):
    """M_p = rho_m0 L^3 / N_p with rho_m0 = Omega_m0 rho_crit (the same
    8 pi G rho_m0 = 3 Omega_m0 H0^2 that normalises the source S)."""
    sim, cos = pv["simulation"], pv["cosmology"]
    mp = cos["omega_m0"] * RHO_CRIT_H2 * sim["box_mpc_h"] ** 3 / sim["particles_per_side"] ** 3
    assert mp == pytest.approx(sim["particle_mass_msun_h"], rel=0.02)


def test_table_speedups(pv):
    t = pv["table_I"]
    assert t["full"] / t["hc_0.24"] == pytest.approx(9.0)
    assert t["full"] / t["hc_0.12"] == pytest.approx(4.5)
    assert t["full"] / t["hc_0.03"] == pytest.approx(1.5)
    assert t["lcdm_cpu_hours"] * t["full"] == pytest.approx(89680.5)


def test_beta_for_the_paper_cosmology(pv, oracle_mod):
    """Eq. (beta) at a = 1 on the LCDM background of the printed cosmology:
    1 + 2 r_c H0 (1 - Omega_m0 / 2)."""
    cos = pv["cosmology"]
    b = oracle_mod.beta_lcdm(1.0, cos["omega_m0"], cos["rc_H0"])
    assert b == pytest.approx(1 + 2 * cos["rc_H0"] * (1 - cos["omega_m0"] / 2), rel=1e-14)
    assert math.isclose(b, 2.731, rel_tol=1e-12)
