"""heget_integrate_step_noalloc (no device allocation inside the library) against heget_integrate_step.

The allocation-free entry point runs the same kernels with the block partial sums in a fixed
device array, and the sampled-helicity mode without the chirality sort.  Both orders evaluate
each event with the same code, and the processes used here run one wave per 64-event group in
both precisions (no cross-wave accumulation), so every output must be bit-identical to the
allocating entry point.  Two calls in a row, the second smaller, check that the reused array
carries nothing over.
"""
import ctypes
import sys

import numpy as np
import pytest

from phasespace import KIN_C2, random_helicities, rambo_uniforms

pytestmark = pytest.mark.gpu

ALPHA_S = 0.118
CUTS = (20.0, 2.5, 0.4)
# (process, precision, sampled helicities): u u > u u g has three chirality patterns, so the
# allocating entry point sorts its events and the allocation-free one does not
CASES = [("g g > g g g", "fp64", False), ("g g > g g g", "mixed", False),
         ("u u > u u g", "fp64", True), ("u u > u u g", "mixed", True), ("u u~ > g g g", "fp64", True)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("spec,precision,sampled", CASES)
def test_noalloc_matches_integrate_step(torch_dev, spec, precision, sampled):
    torch = torch_dev
    from paper_0909_5257_amd import heget
    proc = heget.Process(spec, precision)
    nf = proc.n_ext - 2
    for n, seed in ((50_003, 1), (3_001, 2)):        # second call smaller than the first
        _say(f"[noalloc] {spec} {precision} sampled={sampled} n={n}")
        rs, u = rambo_uniforms(n, nf, KIN_C2, seed=seed)
        rs_d = torch.from_numpy(rs).to("cuda")
        u_d = torch.from_numpy(u).to("cuda")
        hel = torch.from_numpy(random_helicities(n, proc.n_ext, seed=seed)).to("cuda") if sampled else None
        got = heget.integrate_step(proc, rs_d, u_d, ALPHA_S, *CUTS, helicity=hel, noalloc=True)
        ref = heget.integrate_step(proc, rs_d, u_d, ALPHA_S, *CUTS, helicity=hel)
        torch.cuda.synchronize()
        names = ("momenta", "me2", "weight", "sums")
        for name, a, b in zip(names, got, ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.all(np.isfinite(a)), name
            assert np.array_equal(a, b), f"{name} differs: max |diff| {np.max(np.abs(a - b)):.3e}"
        sums = got[3].cpu().numpy()
        _say(f"[noalloc] n={n}: sum f = {sums[0]:.6e} pb, identical to heget_integrate_step")
        assert sums[0] > 0.0


def test_noalloc_size_limit(torch_dev):
    from paper_0909_5257_amd import heget
    proc = heget.Process("g g > g g g", "fp64")
    cuts = heget.Cuts(*CUTS)
    L = heget.lib()
    # above the fixed work space: rejected on the host before any pointer is used
    st = L.heget_integrate_step_noalloc(proc.handle, (1 << 25) + 1, None, None, None, ALPHA_S, ctypes.byref(cuts),
                                        None, None, None, None, None)
    assert st == 1
