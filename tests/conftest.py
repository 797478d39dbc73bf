import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

import pytest  # noqa: E402

import parity_util  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(autouse=True)
def _parity_test_id(request):
    parity_util.set_test(request.node.nodeid)
    yield


def pytest_terminal_summary(terminalreporter):
    """Worst relative-l2 and element-wise ratio per test, against its bar."""
    if not parity_util.RECORD:
        return
    worst = {}
    for tid, tol, l2, mx in parity_util.RECORD:
        w = worst.setdefault(tid, [tol, 0.0, 0.0, 0])
        w[0] = max(w[0], tol)
        w[1] = max(w[1], l2)
        w[2] = max(w[2], mx)
        w[3] += 1
    terminalreporter.write_sep("-", "parity margins (worst per test: l2 ratio, element-wise ratio, bar, checks)")
    for tid, (tol, l2, mx, k) in sorted(worst.items()):
        terminalreporter.write_line(f"{tid}  l2={l2:.3e}  max={mx:.3e}  bar={tol:.0e}  n={k}")
