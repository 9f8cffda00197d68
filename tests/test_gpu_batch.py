"""Fused uneven batches: identical to one-by-one launches, eagerly and as a replayed hipGraph."""
import numpy as np
import pytest

from conftest import cooperative_processes
from phasespace import KIN_C2, generate_events

pytestmark = pytest.mark.gpu

# multi-wave kernels agree with a lone launch to float64 rounding, single-wave ones bit for bit
COOPERATIVE = cooperative_processes()

FUSED = ["u u~ > g g", "u u~ > g g g", "u u~ > g g g g", "u u~ > g g g g g",
         "u u > u u", "u u > u u g", "u u > u u g g", "u u > u u g g g"]


def _same(spec, r, o, what=""):
    import torch
    if spec in COOPERATIVE:
        assert torch.max(torch.abs(o / r - 1.0)).item() < 1e-13, (spec, what)
    else:
        assert torch.equal(r, o), (spec, what)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(torch, seed=7, lo=6, hi=12):
    rng = np.random.default_rng(seed)
    out = []
    for i, spec in enumerate(FUSED):
        n = int(2 ** rng.uniform(lo, hi))
        nf = len(spec.split(">")[1].split())
        out.append((spec, torch.from_numpy(generate_events(n, nf, KIN_C2, seed=seed, stream=i)).to("cuda")))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_individual(torch_dev, precision):
    torch = torch_dev
    from paper_0909_5257_amd.heget import Process, matrix_elements_batch
    inputs = _inputs(torch)
    procs = [Process(s, precision) for s, _ in inputs]
    ref = [p.matrix_elements(x, 0.118) for p, (_, x) in zip(procs, inputs)]
    torch.cuda.synchronize()
    outs = [torch.full((x.shape[0],), -1.0, dtype=torch.float64, device="cuda") for _, x in inputs]
    matrix_elements_batch([(p, x, o) for p, (_, x), o in zip(procs, inputs, outs)], 0.118)
    torch.cuda.synchronize()
    for (spec, _), r, o in zip(inputs, ref, outs):
        _same(spec, r, o)


def test_batch_graph_replays(torch_dev):
    torch = torch_dev
    from paper_0909_5257_amd.heget import Process, matrix_elements_batch
    inputs = _inputs(torch, seed=8)
    procs = [Process(s, "mixed") for s, _ in inputs]
    ref = [p.matrix_elements(x, 0.118) for p, (_, x) in zip(procs, inputs)]
    torch.cuda.synchronize()
    outs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") for _, x in inputs]
    items = [(p, x, o) for p, (_, x), o in zip(procs, inputs, outs)]
    for rep in range(4):
        for o in outs:
            o.fill_(-1.0)                      # the program's own work between replays
        torch.cuda.synchronize()
        matrix_elements_batch(items, 0.118, use_graph=True)
        torch.cuda.synchronize()
        for (spec, _), r, o in zip(inputs, ref, outs):
            _same(spec, r, o, f"replay {rep}")
