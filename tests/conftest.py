import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side oracle checks")


def golden(name):
    return os.path.join(ROOT, "tests", "golden", name)


@pytest.fixture
def golden_path():
    return golden


def cooperative_processes() -> set:
    """Processes whose kernels (either precision) spread one event group's diagram work over
    several waves; they add into the shared colour vector with float64 LDS atomics, so their
    results agree between launches to float64 rounding rather than bit for bit.  The
    generator records the workgroup shape in the header of each generated source."""
    gen = os.path.join(ROOT, "paper_0909_5257_amd", "csrc", "generated")
    out = set()
    for name in sorted(os.listdir(gen)) if os.path.isdir(gen) else []:
        if not name.endswith(".hip"):
            continue
        with open(os.path.join(gen, name)) as f:
            head = f.read(2000)
        spec = re.search(r'for the process "([^"]+)"', head).group(1)
        w = re.search(r"waves per workgroup (\d+) \(float64\) / (\d+) \(mixed\)", head)
        if int(w.group(1)) > 1 or int(w.group(2)) > 1:
            out.add(spec)
    return out
