import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def ref():
    """The C half of the oracle, built on demand."""
    from oracle import build_ref
    if not os.path.exists(build_ref.LIB) or os.path.getmtime(build_ref.LIB) < os.path.getmtime(build_ref.SRC):
        build_ref.build()
    from oracle import ref as r
    return r


def pytest_collection_modifyitems(config, items):
    """Tests marked `slow` take minutes of CPU time; they run only when
    EBC_RUN_SLOW=1 is set."""
    if os.environ.get("EBC_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow CPU test: set EBC_RUN_SLOW=1 to run it")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
