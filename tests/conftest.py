import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size parity case (seconds to minutes)")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Image parity figures of every GPU comparison against the oracle: pixels compared,
    max-abs error on unflagged pixels, the flagged fraction, the largest slack and the
    largest error on a flagged pixel."""
    mod = sys.modules.get("gpu_helpers") or sys.modules.get("tests.gpu_helpers")
    stats = getattr(mod, "PARITY_STATS", None) if mod else None
    if not stats:
        return
    tr = terminalreporter
    tr.section("image parity against the oracle")
    worst_frac = max(s[3] for s in stats)
    tr.write_line(f"{len(stats)} comparisons; worst flagged fraction {worst_frac:.3g}; "
                  f"worst unflagged max-abs {max(s[2] for s in stats):.3g}")
    for test, npx, emax, frac, slack, eflag in stats:
        tr.write_line(f"{test}: {npx} px, unflagged max-abs {emax:.3g}, flagged {frac:.3g}, "
                      f"max slack {slack:.3g}, flagged max-abs {eflag:.3g}")
