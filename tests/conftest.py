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


def load_oracle_sample(name: str) -> dict:
    """A stored oracle sample (tests/golden/oracle_<name>.txt, written by make_oracle_samples.py):
    the workload parameters, the sampled event indices and the oracle's |M|^2 on them."""
    import numpy as np
    meta, rows = {}, []
    with open(golden(f"oracle_{name}.txt")) as f:
        for line in f:
            if line.startswith("# ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                meta[k] = v.strip()
            elif line.strip() and not line.startswith("#"):
                i, v = line.split()
                rows.append((int(i), float(v)))
    return {"spec": meta["spec"], "kin": meta["kinematics"], "n": int(meta["n_events"]), "seed": int(meta["seed"]),
            "stream": int(meta["stream"]), "sha": meta["momenta_sha256"],
            "idx": np.array([r[0] for r in rows], dtype=np.int64), "me2": np.array([r[1] for r in rows])}


def sample_events(sample: dict):
    """Regenerate the whole workload of a stored sample and check that the sampled events are the
    ones the oracle saw (same SHA-256)."""
    import hashlib
    import numpy as np
    from phasespace import KIN_C1, KIN_C2, KIN_C5, generate_events
    kin = {"C1": KIN_C1, "C2": KIN_C2, "C5": KIN_C5}[sample["kin"]]
    nf = len(sample["spec"].split(">")[1].split())
    p = generate_events(sample["n"], nf, kin, seed=sample["seed"], stream=sample["stream"])
    sha = hashlib.sha256(np.ascontiguousarray(p[sample["idx"]]).tobytes()).hexdigest()
    assert sha == sample["sha"], "regenerated events differ from those the oracle evaluated"
    return p


def rel_err_summary(got, ref) -> dict:
    """max, p99 and median relative error (the aggregation of the parity bar is the max)."""
    import numpy as np
    rel = np.abs(np.asarray(got) / np.asarray(ref) - 1.0)
    return {"max": float(rel.max()), "p99": float(np.percentile(rel, 99)), "median": float(np.median(rel)),
            "n": int(rel.size)}
