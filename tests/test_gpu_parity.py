"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: the float64 path agrees with the oracle to 1e-12 maximum relative
error on every compared event, the mixed path (float32 wavefunctions and
amplitudes, float64 JAMP and colour sum) to 1e-5.  Inputs are seeded RAMBO
events of the workloads' kinematics.
"""
import math
import os
import sys

import numpy as np
import pytest

from phasespace import KIN_C1, KIN_C2, KIN_C5, generate_events

pytestmark = pytest.mark.gpu

ALPHA_S = 0.118
TOL = {"fp64": 1e-12, "mixed": 1e-5}

# (process, events compared one by one with the oracle)
SMALL_CASES = [
    ("g g > g g", 200), ("g g > g g g", 131), ("g g > g g g g", 40),
    ("u u~ > g g", 200), ("u u~ > g g g", 131), ("u u~ > g g g g", 80), ("u u~ > g g g g g", 12),
    ("u u > u u", 200), ("u u > u u g", 131), ("u u > u u g g", 80), ("u u > u u g g g", 8),
    ("u g > u g", 200), ("u g > u g g", 131), ("u g > u g g g", 64), ("u u~ > u u~", 200),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _nfinal(spec):
    return len(spec.split(">")[1].split())


def _run(torch, spec, precision, p_np):
    from paper_0909_5257_amd.heget import Process, supported_processes
    if os.environ.get("HEGET_ALLOW_MISSING") == "1" and spec not in supported_processes():
        pytest.skip(f"{spec} not in this build")
    proc = Process(spec, precision)
    p = torch.from_numpy(p_np).to("cuda")
    out = proc.matrix_elements(p, ALPHA_S)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _oracle(spec, p):
    from oracle import oracle_me2
    return oracle_me2(spec, p, ALPHA_S)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("spec,n", SMALL_CASES, ids=[c[0] for c in SMALL_CASES])
def test_parity_small(torch_dev, spec, n, precision):
    kin = KIN_C1 if _nfinal(spec) == 2 else KIN_C2
    p = generate_events(n, _nfinal(spec), kin, seed=0)
    _say(f"[parity] {spec} {precision} n={n}")
    got = _run(torch_dev, spec, precision, p)
    ref = _oracle(spec, p)
    rel = np.abs(got / ref - 1.0)
    _say(f"[parity] {spec} {precision}: max rel err {rel.max():.3e}, median {np.median(rel):.3e}")
    assert np.all(np.isfinite(got))
    assert rel.max() <= TOL[precision]


# stored oracle samples (tests/golden/oracle_<name>.txt): 512 sampled events of each workload-size
# launch (C1, C2, C3 and the metric's u u~ > 5g), and of the serving pools at C5 kinematics
FULL_SIZE = ["gg_gg_c1_65536", "uux_gggg_c2_2e20", "uu_uugg_c2_2e20", "gg_gggg_c2_2e21",
             "uux_ggggg_c2_2e20", "uu_uuggg_c2_2e18"]
SERVING_C5 = ["gg_ggg_c5_2e18", "gg_gggg_c5_2e18", "uux_ggggg_c5_2e18", "uu_uuggg_c5_2e18"]


def _sampled_parity(torch, name):
    from conftest import load_oracle_sample, rel_err_summary, sample_events
    s = load_oracle_sample(name)
    p = sample_events(s)
    for precision in ("fp64", "mixed"):
        _say(f"[sampled] {name} {s['spec']} {precision} n={s['n']}")
        got = _run(torch, s["spec"], precision, p)
        assert np.all(np.isfinite(got)) and np.all(got > 0)
        err = rel_err_summary(got[s["idx"]], s["me2"])
        _say(f"[sampled] {name} {precision}: rel err vs oracle over {err['n']} events: max {err['max']:.3e}, "
             f"p99 {err['p99']:.3e}, median {err['median']:.3e}")
        assert err["max"] <= TOL[precision]


@pytest.mark.parametrize("name", FULL_SIZE)
def test_parity_full_size_sampled(torch_dev, name):
    """Workload-size launches, compared with the oracle on 512 sampled events, both precisions."""
    _sampled_parity(torch_dev, name)


@pytest.mark.parametrize("name", SERVING_C5)
def test_parity_serving_kinematics(torch_dev, name):
    """The serving workload's kinematics (sqrt(s) up to 3 TeV) at 2^18 events, 512 sampled."""
    _sampled_parity(torch_dev, name)


def test_batch_independence_and_ragged_sizes(torch_dev):
    """A point's result does not depend on batch size or position (bit-identical)."""
    spec = "u u~ > g g g"
    p = generate_events(1000, 3, KIN_C2, seed=3)
    full = _run(torch_dev, spec, "fp64", p)
    for lo, hi in [(0, 1), (5, 70), (63, 64), (64, 129), (999, 1000)]:
        part = _run(torch_dev, spec, "fp64", np.ascontiguousarray(p[lo:hi]))
        assert np.array_equal(part, full[lo:hi])


def test_colour_matrix_through_abi(torch_dev):
    from fractions import Fraction
    from oracle.colour import colour_data
    from paper_0909_5257_amd.heget import Process
    for spec in ["g g > g g g", "u u~ > g g g g", "u u > u u g g"]:
        num, den, val = Process(spec).color_matrix()
        ref = colour_data(spec).N_frac
        k = num.shape[0]
        assert all(Fraction(int(num[i, j]), int(den[i, j])) == ref[i][j] for i in range(k) for j in range(k))


def test_abi_argument_errors(torch_dev):
    import ctypes
    torch = torch_dev
    from paper_0909_5257_amd.heget import HegetError, Process, lib
    proc = Process("g g > g g")
    p = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    L = lib()
    h = proc.handle
    assert L.heget_matrix_elements(h, p.data_ptr(), 4, -1.0, out.data_ptr(), None) == 1
    assert L.heget_matrix_elements(h, p.data_ptr(), 4, float("nan"), out.data_ptr(), None) == 1
    assert L.heget_matrix_elements(h, p.data_ptr() + 8, 3, 0.118, out.data_ptr(), None) == 1
    assert L.heget_matrix_elements(h, None, 4, 0.118, out.data_ptr(), None) == 1
    assert L.heget_matrix_elements(h, p.data_ptr(), -1, 0.118, out.data_ptr(), None) == 1
    assert L.heget_matrix_elements(h, None, 0, 0.118, None, None) == 0      # empty batch: nothing queued
    with pytest.raises(HegetError):
        Process("g g > g g g g g g")              # eight gluons: no kernel generated
    with pytest.raises(HegetError):
        Process("g g > t t~")
