"""Test hooks of the C ABI: gauge invariance of the GPU amplitudes and their colour vectors.

* eps -> k: replacing any external gluon's polarisation by its momentum (over its
  energy) must make every helicity amplitude vanish (current conservation of the
  three- and four-gluon and quark-gluon vertices of section 4 with the colour
  factors of section 2.1).  A wrong relative sign or colour coefficient between
  diagram types leaves a remainder of the size of |M|^2.  Bar: the substituted
  |M|^2 is at most 1e-12 (float64) / 1e-5 (mixed) times the unsubstituted one.
* colour vectors: for every evaluated helicity configuration the kernels' reduced
  colour vector y must equal c * M J, with J the oracle's colour-basis amplitudes
  of eq. (color-amplitude) and M the exported exact reduction map, for ONE complex
  c per event and configuration (phase conventions of the external states differ
  between the two implementations; couplings are 1 in the kernels, so
  |c| = g_s^-(n-2)).  This pins the relative phases and sizes of all colour
  components.  And y^H W y must equal the oracle's per-helicity colour sum
  J^H N J (eq. color-averaged-amplitude).
"""
import sys

import numpy as np
import pytest

from phasespace import KIN_C1, KIN_C2, generate_events

pytestmark = pytest.mark.gpu

ALPHA_S = 0.118
TOL = {"fp64": 1e-12, "mixed": 1e-5}

GAUGE_SPECS = ["g g > g g", "g g > g g g", "g g > g g g g", "u u~ > g g", "u u~ > g g g", "u u~ > g g g g",
               "u u > u u g", "u u > u u g g", "u g > u g g", "u g > u g g g"]
JAMP_SPECS = ["g g > g g", "g g > g g g", "g g > g g g g", "u u~ > g g g", "u u~ > g g g g", "u u > u u",
              "u u > u u g", "u u > u u g g", "u g > u g g g", "u u~ > u u~"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _events(spec, n, seed=4):
    nf = len(spec.split(">")[1].split())
    return generate_events(n, nf, KIN_C1 if nf == 2 else KIN_C2, seed=seed)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("spec", GAUGE_SPECS)
def test_gauge_substitution_vanishes(torch_dev, spec, precision):
    torch = torch_dev
    from paper_0909_5257_amd.heget import Process
    proc = Process(spec, precision)
    p = torch.from_numpy(_events(spec, 300)).to("cuda")
    ref, _ = proc.matrix_elements_hook(p, ALPHA_S)
    plain = proc.matrix_elements(p, ALPHA_S)
    torch.cuda.synchronize()
    ref, plain = ref.cpu().numpy(), plain.cpu().numpy()
    assert np.all(ref > 0)
    # the hook kernels are the hot-path kernels plus the switch: same |M|^2 to rounding
    assert np.max(np.abs(ref / plain - 1.0)) < (1e-13 if precision == "fp64" else 1e-5)
    gluons = [i for i, f in enumerate(spec.replace(">", "").split()) if f == "g"]
    worst = 0.0
    for leg in gluons:
        got, _ = proc.matrix_elements_hook(p, ALPHA_S, gauge_leg=leg)
        torch.cuda.synchronize()
        ratio = np.abs(got.cpu().numpy()) / ref
        _say(f"[gauge] {spec} {precision} leg {leg}: max |M|^2(eps->k/E) / |M|^2 = {ratio.max():.3e}")
        worst = max(worst, ratio.max())
    assert worst <= TOL[precision]


@pytest.mark.parametrize("spec", JAMP_SPECS)
def test_colour_vectors_match_oracle_amplitudes(torch_dev, spec):
    torch = torch_dev
    from oracle import oracle_amplitudes
    from oracle.colour import colour_data
    from oracle.me2 import colour_sum
    from paper_0909_5257_amd.heget import Process
    proc = Process(spec, "fp64")
    m_frac, w_frac, slot_hel = proc.colour_reduction()
    n_ext = proc.n_ext
    mmat = np.array([[float(x) for x in row] for row in m_frac])
    wmat = np.array([[float(x) for x in row] for row in w_frac])
    ev = _events(spec, 24, seed=9)
    me2, jamp = proc.matrix_elements_hook(torch.from_numpy(ev).to("cuda"), ALPHA_S, with_jamp=True)
    torch.cuda.synchronize()
    y = jamp.cpu().numpy()
    y = y[..., 0] + 1j * y[..., 1]                                      # [N, S, K']
    hels = np.where((slot_hel[:, None] >> np.arange(n_ext)[None, :]) & 1, 1, -1)
    jo, _ = oracle_amplitudes(spec, ev, ALPHA_S, hels=hels)              # [S, N, K]
    v = np.einsum("ak,snk->nsa", mmat, jo)                              # M J, [N, S, K']
    g = np.sqrt(4.0 * np.pi * ALPHA_S)
    # one complex constant per (event, configuration)
    c = np.einsum("nsa,nsa->ns", v.conj(), y) / np.maximum(np.einsum("nsa,nsa->ns", v.conj(), v).real, 1e-300)
    resid = np.linalg.norm(y - c[..., None] * v, axis=2)
    scale = np.linalg.norm(y, axis=2).max(axis=1, keepdims=True)        # largest configuration of the event
    big = np.linalg.norm(y, axis=2) > 1e-6 * scale
    rel = resid / scale
    _say(f"[jamp] {spec}: {y.shape[1]} configurations x {y.shape[0]} events, K' = {y.shape[2]} of "
         f"{proc.n_colours}: max |y - c M J| / |y|max {rel.max():.3e}; |c| g^(n-2) in "
         f"[{(np.abs(c[big]) * g ** (n_ext - 2)).min():.15f}, {(np.abs(c[big]) * g ** (n_ext - 2)).max():.15f}]")
    assert rel.max() <= 1e-12
    # |c| g^(n-2) = 1: a least-squares constant is off by at most the residual over the vector's own
    # norm, so small configurations of an event carry a proportionally looser bound
    own = np.linalg.norm(y, axis=2)
    dev = np.abs(np.abs(c) * g ** (n_ext - 2) - 1.0)
    bound = 1e-12 + 2.0 * resid / np.maximum(own, 1e-300)
    _say(f"[jamp] {spec}: max ||c| g^(n-2) - 1| {dev[big].max():.3e}, max of it over its bound "
         f"{(dev[big] / bound[big]).max():.3f}")
    assert np.all(dev[big] <= bound[big])
    # per-helicity colour sums: y^H W y g^(2(n-2)) against J^H N J
    q = np.einsum("nsa,ab,nsb->ns", y.conj(), wmat, y).real * g ** (2 * (n_ext - 2))
    qo = colour_sum(jo, colour_data(spec).N).T                          # [N, S]
    tot = qo.sum(axis=1, keepdims=True)
    err = np.abs(q - qo) / tot
    _say(f"[jamp] {spec}: per-configuration colour sums, max |q - q_oracle| / sum {err.max():.3e}")
    assert err.max() <= 1e-12
    # and the configurations add up to the summed entry point (x2 for the flipped partners, x1/4)
    assert np.max(np.abs(0.5 * tot[:, 0] / me2.cpu().numpy() - 1.0)) < 1e-12


def test_hook_errors(torch_dev):
    torch = torch_dev
    from paper_0909_5257_amd.heget import HegetError, Process, lib
    p = torch.from_numpy(_events("u u~ > g g", 8)).to("cuda")
    proc = Process("u u~ > g g", "fp64")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    L = lib()
    assert L.heget_matrix_elements_hook(proc.handle, p.data_ptr(), 8, ALPHA_S, 0, out.data_ptr(), None, None) == 1
    assert L.heget_matrix_elements_hook(proc.handle, p.data_ptr(), 8, ALPHA_S, 4, out.data_ptr(), None, None) == 1
    assert L.heget_matrix_elements_hook(proc.handle, p.data_ptr(), 8, ALPHA_S, -2, out.data_ptr(), None, None) == 1
    assert L.heget_matrix_elements_hook(proc.handle, p.data_ptr(), 8, ALPHA_S, 2, out.data_ptr(), None, None) == 0
    big = Process("u u~ > g g g g g", "fp64")          # seven legs: no test-hook kernels
    with pytest.raises(HegetError):
        big.matrix_elements_hook(torch.zeros((4, 7, 4), dtype=torch.float64, device="cuda"), ALPHA_S)
    torch.cuda.synchronize()
