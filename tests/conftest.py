import os
import sys

import pytest

# The oracle runs OpenMP over elements; under several test workers one
# thread each avoids oversubscribing the host (set before the oracle loads).
if os.environ.get("PYTEST_XDIST_WORKER") and "OMP_NUM_THREADS" not in os.environ:
    os.environ["OMP_NUM_THREADS"] = "1"

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if REPO not in sys.path:
    sys.path.insert(0, REPO)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU run of the oracle")


@pytest.fixture(scope="session")
def O():
    from oracle import oracle

    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_1912_12059_amd import nsk

    nsk.load()
    return nsk


def pytest_terminal_summary(terminalreporter):
    """Print every recorded check: the largest achieved error, its bound and
    their ratio, so the headroom of each tolerance is in the log."""
    tol = sys.modules.get("tolerances")
    if tol is None or not tol.RECORDS:
        return
    tr = terminalreporter
    tr.section("achieved error against its bound")
    tr.write_line(f"{'achieved':>11} {'bound':>11} {'ratio':>8}  quantity / test")
    for (test, q), (a, b) in sorted(tol.RECORDS.items()):
        tr.write_line(f"{a:11.3e} {b:11.3e} {a / b if b else float('nan'):8.2e}  {q} / {test}")
