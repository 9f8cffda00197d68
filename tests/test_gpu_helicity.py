"""Monte Carlo helicity mode: one helicity configuration per event (program structure, section 3.2).

Each event's result must equal the oracle's term of the helicity sum for the drawn
configuration, 1/4 * sum_ab J_a N_ab J_b^*, to the path's tolerance relative to the
event's summed |M|^2 (single helicity terms can be tiny next to the sum); structural
zeros must come out exactly 0; and summing the mode over all 2^n patterns must give the
helicity-summed entry point.
"""
import os
import sys

import numpy as np
import pytest

from phasespace import KIN_C1, KIN_C2, generate_events, random_helicities

pytestmark = pytest.mark.gpu

ALPHA_S = 0.118
TOL = {"fp64": 1e-12, "mixed": 1e-5}
CASES = [
    ("g g > g g", 200), ("g g > g g g", 131), ("g g > g g g g", 40),
    ("u u~ > g g g", 131), ("u u~ > g g g g", 40), ("u u~ > g g g g g", 12),
    ("u u > u u", 200), ("u u > u u g", 131), ("u u > u u g g", 40), ("u u > u u g g g", 8),
    ("u g > u g g", 131), ("u u~ > u u~", 200),
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


def _events(spec, n):
    kin = KIN_C1 if _nfinal(spec) == 2 else KIN_C2
    p = generate_events(n, _nfinal(spec), kin, seed=0)
    h = random_helicities(n, p.shape[1], seed=0)
    return p, h


def _gpu_hel(torch, spec, precision, p_np, h_np):
    from paper_0909_5257_amd.heget import Process, supported_processes
    if os.environ.get("HEGET_ALLOW_MISSING") == "1" and spec not in supported_processes():
        pytest.skip(f"{spec} not in this build")
    proc = Process(spec, precision)
    out = proc.matrix_elements_helicity(torch.from_numpy(p_np).to("cuda"), torch.from_numpy(h_np).to("cuda"),
                                        ALPHA_S)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("spec,n", CASES, ids=[c[0] for c in CASES])
def test_helicity_mode_parity(torch_dev, spec, n, precision):
    from oracle import oracle_me2
    p, h = _events(spec, n)
    _say(f"[helicity] {spec} {precision} n={n}")
    got = _gpu_hel(torch_dev, spec, precision, p, h)
    full, per_hel = oracle_me2(spec, p, ALPHA_S, return_helicities=True)
    ref = 0.25 * per_hel[h, np.arange(n)]
    err = np.abs(got - ref) / full
    _say(f"[helicity] {spec} {precision}: max err / summed |M|^2 {err.max():.3e}")
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL[precision]
    # chirality zeros (the oracle's term is exactly 0 for every event) are exact zeros
    structural = np.all(per_hel == 0.0, axis=1)
    assert np.all(got[structural[h]] == 0.0)


@pytest.mark.parametrize("spec", ["g g > g g g", "u u > u u g", "u g > u g g"])
def test_helicity_mode_sums_to_summed_entry_point(torch_dev, spec):
    from paper_0909_5257_amd.heget import Process
    torch = torch_dev
    n = 67
    p, _ = _events(spec, n)
    n_ext = p.shape[1]
    pt = torch.from_numpy(p).to("cuda")
    for precision in ("fp64", "mixed"):
        proc = Process(spec, precision)
        total = torch.zeros(n, dtype=torch.float64, device="cuda")
        for hh in range(1 << n_ext):
            hel = torch.full((n,), hh, dtype=torch.int32, device="cuda")
            total += proc.matrix_elements_helicity(pt, hel, ALPHA_S)
        summed = proc.matrix_elements(pt, ALPHA_S)
        torch.cuda.synchronize()
        rel = (total / summed - 1.0).abs().max().item()
        _say(f"[helicity] {spec} {precision}: sum over patterns vs summed {rel:.3e}")
        assert rel <= (1e-13 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("spec", ["g g > g g g", "u u > u u g"])
def test_helicity_mode_out_of_range_gives_nan(torch_dev, spec):
    """Single-pattern processes run in event order; two-quark-line processes sort the events by
    chirality pattern first (out-of-range patterns sort last): both leave NaN exactly there."""
    from oracle import oracle_me2
    torch = torch_dev
    p, h = _events(spec, 130)
    n_ext = p.shape[1]
    h = h.copy()
    h[3], h[77], h[129] = -1, 1 << n_ext, 1 << 30
    got = _gpu_hel(torch, spec, "fp64", p, h)
    bad = np.zeros(130, bool)
    bad[[3, 77, 129]] = True
    assert np.all(np.isnan(got[bad]))
    assert np.all(np.isfinite(got[~bad]))
    full, per_hel = oracle_me2(spec, p, ALPHA_S, return_helicities=True)
    idx = np.nonzero(~bad)[0]
    err = np.abs(got[idx] - 0.25 * per_hel[h[idx], idx]) / full[idx]
    assert err.max() <= TOL["fp64"]


def test_helicity_mode_large_batch_two_quark_lines(torch_dev):
    """A batch of 2^16 events of u u > u u g g with drawn patterns (sorted by chirality pattern
    inside the library) against the oracle on sampled events."""
    from oracle import oracle_me2
    torch = torch_dev
    spec = "u u > u u g g"
    n = 1 << 16
    p, h = _events(spec, n)
    got = _gpu_hel(torch, spec, "fp64", p, h)
    idx = np.linspace(0, n - 1, 24).astype(int)
    full, per_hel = oracle_me2(spec, p[idx], ALPHA_S, return_helicities=True)
    err = np.abs(got[idx] - 0.25 * per_hel[h[idx], np.arange(len(idx))]) / full
    _say(f"[helicity] {spec} 2^16 sorted: max err / summed |M|^2 {err.max():.3e}")
    assert err.max() <= TOL["fp64"]
    assert np.all(np.isfinite(got))


def test_helicity_mode_argument_errors(torch_dev):
    import ctypes
    from paper_0909_5257_amd.heget import Process, lib
    proc = Process("g g > g g", "fp64")
    L = lib()
    mom = torch_dev.zeros((4, 4, 4), dtype=torch_dev.float64, device="cuda")
    out = torch_dev.zeros(4, dtype=torch_dev.float64, device="cuda")
    vp = ctypes.c_void_p
    assert L.heget_matrix_elements_helicity(proc.handle, vp(mom.data_ptr()), None, 4, ALPHA_S,
                                            vp(out.data_ptr()), None) == 1
    assert L.heget_matrix_elements_helicity(None, vp(mom.data_ptr()), None, 4, ALPHA_S, vp(out.data_ptr()),
                                            None) == 1
    # zero events queue nothing and succeed with NULL buffers
    assert L.heget_matrix_elements_helicity(proc.handle, None, None, 0, ALPHA_S, None, None) == 0
