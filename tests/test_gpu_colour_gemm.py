"""Colour quadratic form q = J N J^* (eq. color-averaged-amplitude) through the C ABI.

Modes: float64 and float32 on the matrix cores, bf16x3 (bf16 hi/lo split, three matrix-core
products, float32 accumulate), float64 on the vector ALUs.  The references are the oracle's
exact colour matrices and, for the amplitude vectors, the oracle's own colour-basis amplitudes
(g g > g g g g) or seeded random vectors contracted in float64 numpy (the plain definition).
Bars: 1e-12 relative for the two float64 modes, 1e-5 for float32 and bf16x3.
"""
import numpy as np
import pytest

from phasespace import KIN_C2, generate_events

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp64_valu": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5}
MODES = list(TOL)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def oracle_rows():
    from oracle import oracle_amplitudes
    from oracle.colour import colour_data
    spec = "g g > g g g g"
    p = generate_events(6, 4, KIN_C2, seed=0)
    jamp, _ = oracle_amplitudes(spec, p, 0.118)          # [H, N, K]
    nmat = colour_data(spec).N
    j = jamp.reshape(-1, jamp.shape[-1])
    exact = np.einsum("ra,ab,rb->r", j, nmat, j.conj()).real
    keep = exact > 1e-12 * exact.max()                   # drop vanishing helicities
    j = j[keep] / np.sqrt(exact[keep].max())
    exact = exact[keep] / exact[keep].max()
    return nmat, j, exact


def _run(torch, nmat, x, mode):
    from paper_0909_5257_amd.heget import colour_quadratic_form
    q = colour_quadratic_form(torch.from_numpy(nmat).cuda(), torch.from_numpy(x).cuda(), mode)
    torch.cuda.synchronize()
    return q.cpu().numpy()


@pytest.mark.parametrize("mode", MODES)
def test_colour_gemm_modes(torch_dev, oracle_rows, mode):
    nmat, j, exact = oracle_rows
    x = np.stack([j.real, j.imag], axis=1)               # [R, 2, K]
    q = _run(torch_dev, nmat, x, mode)
    rel = np.abs(q / exact - 1.0)
    print(f"[colour-gemm] {mode}: rows {len(exact)}, max rel err {rel.max():.3e}, median {np.median(rel):.3e}",
          flush=True)
    assert rel.max() <= TOL[mode]


# colour matrices of the paper's processes: K = 2 ... 240 (240 is above the hand-written kernels'
# 128 and takes the library-GEMM path); ragged row counts that leave partial tiles
@pytest.mark.parametrize("spec,rows", [("u u~ > g g", 37), ("g g > g g", 1001), ("u u~ > g g g", 515),
                                       ("g g > g g g", 4099), ("u u > u u g g", 999), ("g g > g g g g", 3000),
                                       ("u u > u u g g g", 333)])
@pytest.mark.parametrize("mode", MODES)
def test_colour_gemm_shapes(torch_dev, spec, rows, mode):
    from oracle.colour import colour_data
    nmat = colour_data(spec).N
    k = nmat.shape[0]
    if mode == "fp64_valu" and k > 128:
        pytest.skip("the vector-ALU mode covers K <= 128")
    rng = np.random.default_rng(k * 1000 + rows)
    x = rng.standard_normal((rows, 2, k))
    q = _run(torch_dev, nmat, x, mode)
    ref = np.einsum("rca,ab,rcb->r", x, nmat, x)
    # rounding of a sum is bounded relative to the sum of the magnitudes of its terms (random
    # vectors meet the near-null directions of the singular two-quark-line matrices)
    mag = np.einsum("rca,ab,rcb->r", np.abs(x), np.abs(nmat), np.abs(x))
    err = np.abs(q - ref) / mag
    print(f"[colour-gemm] {spec} K={k} rows={rows} {mode}: max |q - q_ref| / sum|terms| {err.max():.3e}, "
          f"max rel err {np.max(np.abs(q / ref - 1.0)):.3e}", flush=True)
    assert err.max() <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_colour_gemm_workload_size(torch_dev, mode):
    """The C3 workload shape: 2^21 amplitude rows of K = 120 (g g > g g g g), seeded random J;
    512 sampled rows against the float64 definition, and every row finite and positive."""
    from oracle.colour import colour_data
    torch = torch_dev
    from paper_0909_5257_amd.heget import colour_quadratic_form
    nmat = colour_data("g g > g g g g").N
    rows = 1 << 21
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    x = torch.randn((rows, 2, 120), dtype=torch.float64, device="cuda", generator=g)
    q = colour_quadratic_form(torch.from_numpy(nmat).cuda(), x, mode)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(4).choice(rows, 512, replace=False))
    xs = x[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = np.einsum("rca,ab,rcb->r", xs, nmat, xs)
    got = q.cpu().numpy()
    rel = np.abs(got[idx] / ref - 1.0)
    print(f"[colour-gemm] 2^21 x 120 {mode}: sampled max rel err {rel.max():.3e}", flush=True)
    assert np.all(np.isfinite(got)) and np.all(got > 0)
    assert rel.max() <= TOL[mode]
