"""Colour quadratic form as a GEMM in three precisions, against the oracle's exact colour sum."""
import numpy as np
import pytest

from phasespace import KIN_C2, generate_events

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5}


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


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_colour_gemm_modes(oracle_rows, mode):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0909_5257_amd.heget import colour_quadratic_form
    nmat, j, exact = oracle_rows
    x = np.stack([j.real, j.imag], axis=1)               # [R, 2, K]
    q = colour_quadratic_form(torch.from_numpy(nmat).cuda(), torch.from_numpy(x).cuda(), mode)
    torch.cuda.synchronize()
    rel = np.abs(q.cpu().numpy() / exact - 1.0)
    print(f"[colour-gemm] {mode}: rows {len(exact)}, max rel err {rel.max():.3e}, median {np.median(rel):.3e}",
          flush=True)
    assert rel.max() <= TOL[mode]
