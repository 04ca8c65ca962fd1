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


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Adjudicated near-tie positions of every GPU-vs-oracle top-k comparison."""
    try:
        from _parity import SWAPS
    except Exception:
        return
    if not SWAPS:
        return
    tot = sum(v[0] for v in SWAPS.values())
    res = sum(v[1] for v in SWAPS.values())
    terminalreporter.write_sep("-", f"adjudicated near-tie positions: {tot} of {res} compared")
    for name, (s, n) in sorted(SWAPS.items()):
        if s:
            terminalreporter.write_line(f"{s:6d} / {n:8d}  {name}")
