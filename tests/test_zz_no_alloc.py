"""ndgp_residual_noalloc: the residual with the library's static device scratch
(no workspace, no allocation, no synchronisation) against ndgp_residual with a
workspace, through the C ABI: the same bits for r and the relative norm, on
two calls in a row with the second on a smaller level, on a patch level, and
on a side stream; levels above NDGP_NOALLOC_MAX_CELLS are refused."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1511_08200_amd import ndgp, synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ndgp.lib()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def both(grid, params, deltas, phi, level, stream=None):
    r_ref, rel_ref = ndgp.residual(grid, params, deltas, phi, level=level)
    n = grid.level_n(level)
    r = torch.full((n,) * 3, np.nan, dtype=torch.float64, device="cuda")
    norms = torch.full((3,), np.nan, dtype=torch.float64, device="cuda")
    if stream is None:
        ndgp.residual_noalloc(grid, params, deltas, phi, level=level, r_out=r, norms=norms)
    else:
        with torch.cuda.stream(stream):
            ndgp.residual_noalloc(grid, params, deltas, phi, level=level, r_out=r, norms=norms,
                                  stream=stream)
        stream.synchronize()
    torch.cuda.synchronize()
    return r_ref, rel_ref, r, norms.cpu().numpy()


def test_noalloc_residual_equals_workspace_residual():
    rng = np.random.default_rng(3)
    params = ndgp.Params(rc=2.0)
    # first call: 64^3 domain (several reduction and tile blocks)
    f = synth.make_field(64, 2.0, 81, n_tophats=5)
    grid = ndgp.Grid(n=64, h=ndgp.cell_size(64.0, 64))
    phi = dev(rng.standard_normal((64,) * 3) * 1e-7)
    r_ref, rel_ref, r, norms = both(grid, params, [dev(f.delta)], phi, 0)
    print(f"64^3: rel {rel_ref:.6e} noalloc {norms[2]:.6e}", flush=True)
    assert torch.equal(r, r_ref)
    assert norms[2] == rel_ref
    assert norms[0] > 0 and norms[1] > 0
    # second call, smaller: 16^3 domain; stale scratch from the first call must not leak in
    f2 = synth.make_field(16, 1.0, 82)
    grid2 = ndgp.Grid(n=16, h=ndgp.cell_size(16.0, 16))
    phi2 = dev(rng.standard_normal((16,) * 3) * 1e-7)
    r_ref, rel_ref, r, norms = both(grid2, params, [dev(f2.delta)], phi2, 0)
    print(f"16^3: rel {rel_ref:.6e} noalloc {norms[2]:.6e}", flush=True)
    assert torch.equal(r, r_ref)
    assert norms[2] == rel_ref
    # a patch level (ghost shell as boundary) on a side stream
    o = (4, 20, 9)
    d1 = synth.patch_delta(f2, 16, [o], 16)
    gridp = ndgp.Grid(n=16, h=ndgp.cell_size(16.0, 16), patches=[ndgp.Patch(16, o)])
    phip = dev(rng.standard_normal((18,) * 3) * 1e-8)
    side = torch.cuda.Stream()
    r_ref, rel_ref, r, norms = both(gridp, params, [dev(f2.delta), dev(d1)], phip, 1, stream=side)
    assert torch.equal(r, r_ref)
    assert norms[2] == rel_ref
    # r_out is optional
    norms_only = torch.empty(3, dtype=torch.float64, device="cuda")
    ndgp.residual_noalloc(grid2, params, [dev(f2.delta)], phi2, norms=norms_only)
    torch.cuda.synchronize()
    assert norms_only[2].item() == ndgp.residual(grid2, params, [dev(f2.delta)], phi2)[1]


def test_noalloc_residual_refuses_levels_above_its_scratch():
    n = 256
    grid = ndgp.Grid(n=n, h=ndgp.cell_size(256.0, n))
    d = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(ndgp.NdgpError) as e:
        ndgp.residual_noalloc(grid, ndgp.Params(rc=1.0), [d], d)
    assert e.value.status == ndgp.NDGP_EINVAL
    assert "NDGP_NOALLOC_MAX_CELLS" in str(e.value)
