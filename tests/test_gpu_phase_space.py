"""Device RAMBO, jet cuts and integration step against the oracle (through the C ABI).

Bars: momenta to 1e-13 * k of sqrt(s) (absolute), with k = max(1, gamma^2) of the event's
RAMBO boost (the two implementations' log/sin/cos differ in the last bit, and the boost of
nearly collinear draws amplifies that by up to gamma^2); phase-space weights to 1e-14
relative; cut flags identical except for events whose cut variables sit within 1e-9
(relative) of a threshold; the chained |M|^2 and event weights to 1e-11 * k relative to the
event's helicity-summed value; the sums of f and f^2 to 1e-10 and bit-identical between runs.
"""
import ctypes
import sys

import numpy as np
import pytest

from phasespace import KIN_C1, KIN_C2, random_helicities, rambo_massless, rambo_uniforms

pytestmark = pytest.mark.gpu

ALPHA_S = 0.118
CUTS = (20.0, 2.5, 0.4)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cuda(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("nf", [2, 3, 4, 5, 6, 7, 8])
def test_rambo_parity(torch_dev, nf):
    from oracle import phase_space as ops
    from paper_0909_5257_amd import heget
    n = 1000 + nf
    rs, u = rambo_uniforms(n, nf, KIN_C2, seed=nf)
    _say(f"[rambo] n_final={nf} n={n}")
    mom, w = heget.rambo(_cuda(torch_dev, rs), _cuda(torch_dev, u))
    torch_dev.cuda.synchronize()
    ref_m, ref_w = ops.rambo(rs, u)
    k = np.maximum(1.0, ops.rambo_gamma(u) ** 2)
    dev = np.abs(mom.cpu().numpy() - ref_m).max(axis=(1, 2))
    _say(f"[rambo] max |dp| / (k sqrt s) = {np.max(dev / (k * rs)):.2e}, max k = {k.max():.1f}")
    assert np.all(dev <= 1e-13 * k * rs)
    np.testing.assert_allclose(w.cpu().numpy(), ref_w, rtol=1e-14)


class _Fixed:
    def __init__(self, u):
        self.u = u

    def random(self, shape):
        return self.u


@pytest.mark.parametrize("nf,dr", [(2, 0.0), (3, 0.4), (5, 0.4), (5, 0.0)])
def test_cuts_parity(torch_dev, nf, dr):
    from oracle import phase_space as ops
    from paper_0909_5257_amd import heget
    n = 4000
    rs, u = rambo_uniforms(n, nf, KIN_C2, seed=40 + nf)
    fin = rambo_massless(_Fixed(u), nf, rs)          # momenta from the input generator, no cut applied
    mom = np.zeros((n, nf + 2, 4))
    mom[:, 0] = np.stack([rs / 2, 0 * rs, 0 * rs, rs / 2], 1)
    mom[:, 1] = np.stack([rs / 2, 0 * rs, 0 * rs, -rs / 2], 1)
    mom[:, 2:] = fin
    got = heget.apply_cuts(_cuda(torch_dev, mom), *CUTS[:2], dr).cpu().numpy()
    ref = np.array([ops.passes_cuts(p[2:], CUTS[0], CUTS[1], dr) for p in mom])
    tie = np.array([ops.cut_margin(p[2:], CUTS[0], CUTS[1], dr) < 1e-9 for p in mom])
    _say(f"[cuts] n_final={nf} dR={dr}: pass {ref.mean():.3f}, ties {tie.sum()}")
    assert 0 < ref.sum() < n
    assert np.array_equal(got[~tie].astype(bool), ref[~tie])


@pytest.mark.parametrize("spec,n,sampled,precision", [
    ("g g > g g", 3000, False, "fp64"), ("g g > g g g", 1000, False, "fp64"), ("u u~ > g g g g", 300, False, "fp64"),
    ("u u > u u g", 1000, False, "fp64"), ("g g > g g g", 1000, True, "fp64"), ("u u > u u g g", 200, True, "fp64"),
    ("g g > g g g g", 300, False, "mixed"), ("g g > g g g", 1000, False, "mixed"),
    ("u u > u u g g", 200, True, "mixed"), ("g g > g g g g", 300, True, "mixed"),
])
def test_integrate_step_parity(torch_dev, spec, n, sampled, precision):
    """Against the oracle's RAMBO, |M|^2 and weights on the same uniforms: 1e-11 (float64, relative to
    |M|^2 times the RAMBO conditioning factor) and 1e-5 (mixed)."""
    from oracle import oracle_me2
    from oracle import phase_space as ops
    from paper_0909_5257_amd import heget
    torch = torch_dev
    nf = len(spec.split(">")[1].split())
    kin = KIN_C1 if nf == 2 else KIN_C2
    dr = 0.0 if nf == 2 else CUTS[2]
    rs, u = rambo_uniforms(n, nf, kin, seed=7)
    hel = random_helicities(n, nf + 2, seed=7) if sampled else None
    _say(f"[integrate] {spec} {precision} n={n} sampled={sampled}")
    proc = heget.Process(spec, precision)
    tol = 1e-11 if precision == "fp64" else 1e-5
    out = heget.integrate_step(proc, _cuda(torch, rs), _cuda(torch, u), ALPHA_S, CUTS[0], CUTS[1], dr,
                               helicity=None if hel is None else _cuda(torch, hel))
    mom, me2, w, sums = (t.cpu().numpy() for t in out)
    again = heget.integrate_step(proc, _cuda(torch, rs), _cuda(torch, u), ALPHA_S, CUTS[0], CUTS[1], dr,
                                 helicity=None if hel is None else _cuda(torch, hel))[3].cpu().numpy()
    torch.cuda.synchronize()
    from conftest import cooperative_processes
    if spec in cooperative_processes():
        # several waves add into one colour vector with float64 LDS atomics in run-dependent order
        assert np.max(np.abs(again / sums - 1.0)) < 1e-13
    else:
        assert np.array_equal(sums, again)

    ref_mom, _ = ops.rambo(rs, u)
    k = np.maximum(1.0, ops.rambo_gamma(u) ** 2)
    assert np.all(np.abs(mom - ref_mom).max(axis=(1, 2)) <= 1e-13 * k * rs)
    mult = float(1 << (nf + 2)) if sampled else 1.0
    if sampled:
        full, per_hel = oracle_me2(spec, ref_mom, ALPHA_S, return_helicities=True)
        ref_me2 = 0.25 * per_hel[hel, np.arange(n)]
        scale = full
    else:
        ref_me2 = oracle_me2(spec, ref_mom, ALPHA_S)
        scale = ref_me2
    ref_f = ops.event_weights(spec, ref_mom, ref_me2 * mult, CUTS[0], CUTS[1], dr)
    f_scale = ops.event_weights(spec, ref_mom, scale * mult, CUTS[0], CUTS[1], dr)
    tie = np.array([ops.cut_margin(p[2:], CUTS[0], CUTS[1], dr) < 1e-9 for p in ref_mom])
    assert not tie.any()
    err = np.abs(me2 - ref_me2) / (scale * k)
    _say(f"[integrate] {spec}: max |d me2| / (k |M|^2) = {err.max():.2e}")
    assert err.max() <= tol
    passed = ref_f != 0
    assert np.array_equal(w != 0, passed)
    assert np.all(np.abs(w - ref_f)[passed] <= tol * (k * f_scale)[passed])
    np.testing.assert_allclose(sums, [ref_f.sum(), (ref_f ** 2).sum()], rtol=10 * tol)
    mean = sums[0] / n
    err = np.sqrt(max(sums[1] / n - mean * mean, 0.0) / (n - 1))
    _say(f"[integrate] {spec}: sigma-hat = {mean:.6g} +- {err:.2g} pb, pass {passed.mean():.3f}")


def test_phase_space_argument_errors(torch_dev):
    from paper_0909_5257_amd import heget
    L = heget.lib()
    cuts = heget.Cuts(20.0, 0.0, 0.4)            # eta_max <= 0 is rejected
    assert L.heget_apply_cuts(6, 10, 1, ctypes.byref(cuts), 1, None) == 1
    assert L.heget_rambo(1, 10, 1, 1, 1, None, None) == 1
    assert L.heget_rambo(9, 10, 1, 1, 1, None, None) == 1
    assert L.heget_rambo(4, 0, None, None, None, None, None) == 0
    proc = heget.Process("g g > g g", "fp64")
    ok = heget.Cuts(20.0, 2.5, 0.0)
    assert L.heget_integrate_step(proc.handle, 0, 1, 1, None, ALPHA_S, ctypes.byref(ok), 16, 1, 1, 1, None) == 1
