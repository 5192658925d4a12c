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
    """Append measured parity figures to gpurun_out/parity_report.jsonl (when
    that directory exists) so runs on the GPU machine leave a record."""
    import json
    import time
    path = os.path.join(ROOT, "gpurun_out", "parity_report.jsonl")

    def _rep(kind, **kw):
        rec = {"test": request.node.nodeid, "kind": kind, "time": time.time(), **kw}
        print(json.dumps(rec, default=float), flush=True)
        if os.path.isdir(os.path.dirname(path)):
            with open(path, "a") as f:
                f.write(json.dumps(rec, default=float) + "\n")
    return _rep
