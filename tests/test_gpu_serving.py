"""Continuous-batching server: results identical alone and in the mix, admission by HBM budget."""
import numpy as np
import pytest

from conftest import cooperative_processes
from phasespace import KIN_C5, generate_events

pytestmark = pytest.mark.gpu

SPECS = ["g g > g g g", "u u~ > g g g g", "u u > u u g g", "g g > g g g g"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pool():
    out = {}
    for i, s in enumerate(SPECS):
        nf = len(s.split(">")[1].split())
        out[s] = generate_events(5000, nf, KIN_C5, seed=11, stream=i)
    return out


def _alone(torch, spec, mom, precision):
    from paper_0909_5257_amd.heget import Process
    p = torch.from_numpy(mom).to("cuda")
    r = Process(spec, precision).matrix_elements(p, 0.118)
    torch.cuda.synchronize()
    return r.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_same_alone_and_served(torch_dev, precision):
    from paper_0909_5257_amd.serving import Server, latency_summary, run_poisson
    pool = _pool()
    rng0 = np.random.default_rng(3)

    def workload(rng):
        spec = SPECS[rng.integers(len(SPECS))]
        n = int(2 ** rng.uniform(8, 12))
        lo = int(rng.integers(0, 5000 - n))
        return spec, pool[spec][lo:lo + n]

    server = Server(SPECS, precisions=(precision,), hbm_budget_bytes=2 << 20, n_streams=4)
    reqs, wall = run_poisson(server, workload, rate_hz=2000.0, n_requests=40, seed=int(rng0.integers(1 << 30)),
                             precision=precision)
    assert all(r.error is None for r in reqs)
    coop = cooperative_processes()
    for r in reqs:
        ref = _alone(torch_dev, r.spec, r.momenta, precision)
        if r.spec in coop:      # multi-wave kernel: float64 LDS atomics in any order
            assert np.max(np.abs(r.result / ref - 1.0)) < 1e-13, (r.rid, r.spec)
        else:
            assert np.array_equal(r.result, ref), (r.rid, r.spec)
    s = latency_summary(reqs)
    print(f"[serving] {precision}: {s}", flush=True)
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_admission_and_oversize_isolation(torch_dev):
    from paper_0909_5257_amd.serving import Server
    pool = _pool()
    spec = "u u~ > g g g g"
    one = pool[spec][:1000]
    budget = int(1.5 * (one.nbytes + 8 * 1000))       # room for one request at a time
    server = Server([spec], precisions=("fp64",), hbm_budget_bytes=budget, n_streams=4)
    reqs = [server.submit(spec, one, "fp64") for _ in range(3)]
    big = server.submit(spec, pool[spec], "fp64")               # does not fit the budget at all
    peak = 0
    while not server.idle():
        server.step()
        peak = max(peak, len(server.running))
    assert peak == 1                                   # admission held the budget
    assert big.error is not None and big.result is None
    ref = _alone(torch_dev, spec, one, "fp64")
    for r in reqs:
        assert r.error is None
        if spec in cooperative_processes():
            assert np.max(np.abs(r.result / ref - 1.0)) < 1e-13
        else:
            assert np.array_equal(r.result, ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_results_against_oracle(torch_dev, precision):
    """Requests of the serving workload (the four processes, C5 kinematics up to 3 TeV, sizes
    2^U[8,12]) are windows of the 2^18-event pools whose sampled events have stored oracle values
    (tests/golden/oracle_*_c5_2e18.txt); every served result at a sampled event is compared."""
    from conftest import load_oracle_sample, rel_err_summary, sample_events
    from paper_0909_5257_amd.serving import Server, run_poisson
    names = {"g g > g g g": "gg_ggg_c5_2e18", "g g > g g g g": "gg_gggg_c5_2e18",
             "u u~ > g g g g g": "uux_ggggg_c5_2e18", "u u > u u g g g": "uu_uuggg_c5_2e18"}
    stored = {spec: load_oracle_sample(name) for spec, name in names.items()}
    pools = {spec: sample_events(s) for spec, s in stored.items()}
    specs = list(names)
    windows = {}

    def window(rng):
        spec = specs[rng.integers(len(specs))]
        s = stored[spec]
        n = int(2 ** rng.uniform(8, 12))
        j = int(rng.integers(len(s["idx"])))
        lo = int(min(max(s["idx"][j] - rng.integers(n), 0), s["n"] - n))
        return spec, lo, n

    server = Server(specs, precisions=(precision,), hbm_budget_bytes=64 << 20, n_streams=4)
    rng = np.random.default_rng(5)
    items = [window(rng) for _ in range(60)]
    reqs = [server.submit(spec, pools[spec][lo:lo + n], precision) for spec, lo, n in items]
    server.drain()
    got_all, ref_all = [], []
    for r, (spec, lo, n) in zip(reqs, items):
        assert r.error is None
        s = stored[spec]
        sel = (s["idx"] >= lo) & (s["idx"] < lo + n)
        assert sel.any()
        got_all.append(r.result[s["idx"][sel] - lo])
        ref_all.append(s["me2"][sel])
    err = rel_err_summary(np.concatenate(got_all), np.concatenate(ref_all))
    print(f"[serving vs oracle] {precision}: {err['n']} sampled events in {len(reqs)} requests: max rel err "
          f"{err['max']:.3e}, p99 {err['p99']:.3e}, median {err['median']:.3e}", flush=True)
    assert err["max"] <= (1e-12 if precision == "fp64" else 1e-5)


def test_failed_request_is_isolated(torch_dev):
    """A request whose launch raises (momenta of the wrong shape for the process) fails alone; its
    stream slot and budget are returned and the others complete."""
    from paper_0909_5257_amd.serving import Server
    pool = _pool()
    spec = "g g > g g g"
    server = Server([spec], precisions=("fp64",), hbm_budget_bytes=64 << 20, n_streams=2)
    good1 = server.submit(spec, pool[spec][:300], "fp64")
    bad = server.submit(spec, pool["g g > g g g g"][:300], "fp64")     # six legs for a five-leg process
    good2 = server.submit(spec, pool[spec][300:700], "fp64")
    server.drain()
    assert bad.error is not None and bad.result is None and bad.done.is_set()
    for r, lo, hi in ((good1, 0, 300), (good2, 300, 700)):
        assert r.error is None
        ref = _alone(torch_dev, spec, pool[spec][lo:hi], "fp64")
        assert np.max(np.abs(r.result / ref - 1.0)) < 1e-13
    assert server.in_use == 0 and sorted(server.free_streams) == [0, 1]
