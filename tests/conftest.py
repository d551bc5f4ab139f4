import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_terminal_summary(terminalreporter):
    """Worst parity error of each GPU-vs-oracle comparison that ran."""
    try:
        from parity import SUMMARY
    except ImportError:
        return
    if not SUMMARY:
        return
    tr = terminalreporter
    tr.section("parity summary (max over fields and interior points)")
    tr.write_line(f"{'case':58s} {'e_gpu':>9s} {'e_oracle64':>10s} {'e_gpu/tol':>9s}")
    for case, eg, ec, r in SUMMARY:
        tr.write_line(f"{case[:58]:58s} {eg:9.2e} {ec:10.2e} {r:9.3f}")
