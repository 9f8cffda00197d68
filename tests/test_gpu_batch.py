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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_c4_batch_against_oracle(torch_dev, precision):
    """The fused uneven batch of the C4 configuration (eight processes, 2^U[10,20] events each from
    seed 7, about 1.6 M events), eager and as a replayed graph, against stored oracle values of 64
    sampled events per process (tests/golden/oracle_fused_c4_<i>.txt)."""
    torch = torch_dev
    from conftest import load_oracle_sample, rel_err_summary, sample_events
    from paper_0909_5257_amd.heget import Process, matrix_elements_batch
    samples = [load_oracle_sample(f"fused_c4_{i}") for i in range(len(FUSED))]
    assert [s["spec"] for s in samples] == FUSED
    xs = [torch.from_numpy(sample_events(s)).to("cuda") for s in samples]
    procs = [Process(s["spec"], precision) for s in samples]
    outs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") for x in xs]
    items = list(zip(procs, xs, outs))
    for graph in (False, True, True):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        matrix_elements_batch(items, 0.118, use_graph=graph)
        torch.cuda.synchronize()
        for s, o in zip(samples, outs):
            got = o.cpu().numpy()
            assert np.all(np.isfinite(got)) and np.all(got > 0), s["spec"]
            err = rel_err_summary(got[s["idx"]], s["me2"])
            print(f"[fused c4] {precision} graph={graph} {s['spec']} ({s['n']} events): max rel err "
                  f"{err['max']:.3e}, p99 {err['p99']:.3e}, median {err['median']:.3e}", flush=True)
            assert err["max"] <= (1e-12 if precision == "fp64" else 1e-5)


def test_graph_cache_after_handle_reuse(torch_dev):
    """A cached batch graph must not survive its handle: destroy a handle after a graph replay and
    create one of the other precision (the allocator tends to hand back the same addresses); the
    next graph call on the same buffers must run the new handle's kernels."""
    torch = torch_dev
    from paper_0909_5257_amd.heget import Process, matrix_elements_batch
    spec = "u u~ > g g g"
    x = torch.from_numpy(generate_events(3000, 3, KIN_C2, seed=12)).to("cuda")
    out = torch.empty(3000, dtype=torch.float64, device="cuda")
    ref = {}
    for precision in ("mixed", "fp64"):
        p = Process(spec, precision)
        ref[precision] = p.matrix_elements(x, 0.118).clone()
        matrix_elements_batch([(p, x, out)], 0.118, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out, ref[precision]), precision
        del p
    # the two precisions differ, so a stale graph would have been caught above
    assert not torch.equal(ref["mixed"], ref["fp64"])
