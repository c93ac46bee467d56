"""The named workloads (CPU: grids, parameters and inputs, no solve)."""
from __future__ import annotations

import numpy as np
import pytest

pytest.importorskip("torch")

from paper_1511_08200_amd import ndgp, presets, synth  # noqa: E402


def test_every_name_loads_without_drawing_its_input():
    for name in presets.NAMES:
        w = presets.load(name)
        assert w.name == name
        if name != "serving":
            assert w._field is None  # drawn on first use only
    with pytest.raises(KeyError):
        presets.load("periodic-1024")


@pytest.mark.parametrize("name,n,box,levels", [("periodic-32", 32, 64.0, 3),
                                                ("periodic-256", 256, 256.0, 6),
                                                ("periodic-512", 512, 512.0, 7)])
def test_periodic_grids(name, n, box, levels):
    w = presets.load(name, rc=5.0, precision=ndgp.PREC_MIXED)
    assert w.grid.n == n and w.grid.patches == []
    assert w.grid.h == ndgp.cell_size(box, n)
    assert w.params.rc == 5.0 and w.params.tol == 1e-10
    assert w.params.precision == ndgp.PREC_MIXED
    # the default hierarchy coarsens to 8^3
    assert int(np.log2(n // 8)) + 1 == levels


def test_small_input_is_the_seeded_field():
    w = presets.load("periodic-32")
    d = w.deltas()
    assert len(d) == 1 and d[0].shape == (32, 32, 32)
    assert np.array_equal(d[0], synth.make_field(32, 1.0, 1512).delta)
    assert abs(float(d[0].mean())) < 1e-12


def test_nested_refinements_sit_on_the_largest_top_hat():
    """The placement drawn from the top-hats alone equals the one computed
    from the whole field, and each refinement lies inside its parent."""
    w = presets.load("nested-256-deep", mode=ndgp.MODE_TRUNCATED, trunc_level=2)
    assert w.params.mode == ndgp.MODE_TRUNCATED and w.params.trunc_level == 2
    f = w.field
    c = synth.densest_tophat_centre(f)
    for q, p in enumerate(w.grid.patches):
        assert p.n == 128
        o = synth.patch_origin_centred(c, 64)
        if q > 0:
            o = tuple(min(max(v, 8), 128 - 64 - 8) for v in o)
            assert all(8 <= v <= 56 for v in p.origin)
        assert p.origin == o
        c = tuple((c[a] - o[a]) * 2 for a in range(3))
    two = presets.load("nested-256")
    assert two.grid.patches == w.grid.patches[:2]


def test_serving_stream():
    w = presets.load("serving")
    assert len(w.trace) == 2000 and w.budget_bytes == 64e9 and w.max_active == 16
    assert {r.n for r in w.trace} == {32, 64, 128, 256}
    assert {r.rc for r in w.trace} == {0.5, 1.0, 2.0, 5.0}
    assert all(1.0 <= r.sigma <= 2.5 for r in w.trace)
    gaps = np.diff([r.arrival for r in w.trace])
    assert np.all(gaps >= 0) and abs(1.0 / gaps.mean() - 50.0) < 5.0
