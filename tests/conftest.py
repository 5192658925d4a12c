import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    yield


@pytest.fixture
def report(request):
    """Print measured parity figures as JSON lines, and append them to the file
    named by SD7_PARITY_REPORT when that variable is set."""
    import json
    import time
    path = os.environ.get("SD7_PARITY_REPORT")

    def _rep(kind, **kw):
        rec = {"test": request.node.nodeid, "kind": kind, "time": time.time(), **kw}
        print(json.dumps(rec, default=float), flush=True)
        if path:
            os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
            with open(path, "a") as f:
                f.write(json.dumps(rec, default=float) + "\n")
    return _rep
