"""The workspace guard bands (NDGP_GUARD_BANDS, on for the test session) make
every workspace larger than without them; the library reads
the variable once per process."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import sys
sys.path.insert(0, %r)
from paper_1511_08200_amd import ndgp
g = ndgp.Grid(n=64, h=1e-3, patches=[ndgp.Patch(32, (8, 8, 8))])
print(ndgp.workspace_bytes(g, ndgp.Params(rc=1.0)))
""" % ROOT


def _bytes(flag):
    env = dict(os.environ, NDGP_GUARD_BANDS=flag)
    out = subprocess.run([sys.executable, "-c", PROBE], capture_output=True, text=True, env=env,
                         check=True)
    return int(out.stdout.strip())


def test_guard_bands_enlarge_the_workspace():
    plain, guarded = _bytes("0"), _bytes("1")
    assert guarded > plain
    assert guarded - plain >= 20 * 256  # a band after each of the dozens of arrays
    assert os.environ.get("NDGP_GUARD_BANDS") == "1"
