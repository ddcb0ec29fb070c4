import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def pytest_sessionfinish(session, exitstatus):
    """With RS_MARGINS_OUT set, write the largest error / bound ratio seen per
    compared quantity by the GPU parity tests (JSON)."""
    out = os.environ.get("RS_MARGINS_OUT")
    h = sys.modules.get("gpu_harness")
    if out and h is not None and h.MARGINS:
        import json
        with open(out, "w") as f:
            json.dump(dict(sorted(h.MARGINS.items())), f, indent=1)
