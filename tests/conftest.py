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
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


def pytest_terminal_summary(terminalreporter):
    """The tightest gradient comparisons of the session (GPU parity runs)."""
    mod = sys.modules.get("_gpu_util")
    margins = getattr(mod, "GRAD_MARGINS", None) if mod else None
    if not margins:
        return
    terminalreporter.write_line(f"gradient parity: {len(margins)} comparisons; tightest (worst element / bound, "
                                f"rel-L2 / bar):")
    for name, worst, l2 in sorted(margins, key=lambda m: -max(m[1], m[2]))[:6]:
        terminalreporter.write_line(f"  {name}: {worst:.3f}, {l2:.3f}")
