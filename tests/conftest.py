import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Every solve in the tests lays out its workspace with guard bands after each
# sub-buffer and checks them when it ends (the library's debugging aid): a
# kernel that writes past its array fails the call.  Set before the library
# is loaded, which reads it once.
os.environ.setdefault("NDGP_GUARD_BANDS", "1")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.lib()
    return O
