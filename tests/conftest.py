import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The launch shapes this session's plans tune go to a file of its own: the
# test processes run oracle sums and many plans between tunings, and shapes
# picked there are not to be reused by other programs (bench.py tunes in
# its own process).
os.environ.setdefault("PF_AUTOTUNE_CACHE",
                      os.path.join(tempfile.gettempdir(), "pf_autotune_tests_%d.json" % os.getpid()))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    return oracle
