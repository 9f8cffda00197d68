"""Pins of the FP64 oracle against things fixed by the paper and by QCD itself.

None of these tests compares the oracle with itself: each checks a value the
paper prints (Tables 1 and 3, the colour statistics of section 3.3), a
textbook closed form, an exact symmetry, or an independent algorithm.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle_me2, oracle_amplitudes
from oracle import lorentz as L
from oracle.berends_giele import bg_amplitudes, bg_quark_amplitudes, trace_word_to_bg
from oracle.colour import (all_assignments, basis_tensor_all, colour_basis, colour_data,
                           diagram_colour_values)
from oracle.me2 import _evaluate, _externals, helicity_table
from oracle.process import enumerate_diagrams, fermion_sign, parse_process
from phasespace import KIN_C1, KIN_C2, generate_events

from conftest import golden

ALPHA_S = 0.118
G2 = 4.0 * math.pi * ALPHA_S


def _table(name):
    rows = []
    for line in open(golden(name)):
        if line.strip() and not line.startswith("#"):
            rows.append([x.strip() for x in line.split("|")])
    return rows


def _minkowski(x):
    return x[..., 0] ** 2 - (x[..., 1:] ** 2).sum(-1)


def _events(spec, n, seed=0, kin=KIN_C2):
    nf = len(spec.split(">")[1].split())
    return generate_events(n, nf, kin, seed=seed)


# ------------------------------------------------------------------ Table 1 / 3

@pytest.mark.parametrize("row", _table("paper_table1.txt"), ids=lambda r: r[0])
def test_table1_diagram_and_colour_counts(row):
    spec, nd, nc = row[0], int(row[1]), int(row[2])
    proc = parse_process(spec)
    assert len(enumerate_diagrams(proc)) == nd
    assert len(colour_basis(proc)) == nc


@pytest.mark.parametrize("row", [r for r in _table("paper_table3.txt") if r[0] != "g g > g g g g g"],
                         ids=lambda r: r[0])
def test_table3_distinct_colour_matrix_values(row):
    spec, nv = row[0], int(row[1])
    cd = colour_data(spec)
    assert cd.distinct_nonzero() == nv
    # N is a Gram matrix: symmetric and positive semi-definite
    assert np.allclose(cd.N, cd.N.T, atol=0)
    assert np.linalg.eigvalsh(cd.N).min() > -1e-12


def test_mc_colour_statistics_gg_4g():
    want = {r[0]: (float(r[1]), float(r[2])) for r in _table("paper_mc_colour.txt")}
    proc = parse_process("g g > g g g g")
    nz = np.abs(basis_tensor_all(proc, colour_basis(proc))) > 1e-12
    f_one, tol = want["fraction_nonzero_per_basis_vector"]
    assert abs(nz[:, 0].mean() - f_one) < tol
    assert abs(nz.mean() - f_one) < tol
    f_all, tol = want["fraction_all_basis_vectors_zero"]
    assert abs((~nz.any(axis=1)).mean() - f_all) < tol


def test_gg_gg_colour_matrix_values():
    """Un-averaged N for four gluons: 19/6 diagonal, -1/3 and 2/3 off it."""
    from fractions import Fraction
    cd = colour_data("g g > g g")
    vals = {cd.N_frac[i][j] * 64 for i in range(6) for j in range(6)}
    assert vals == {Fraction(19, 6), Fraction(-1, 3), Fraction(2, 3)}


# ------------------------------------------------------------ closed forms

def _mandelstam(p):
    s = _minkowski(p[:, 0] + p[:, 1])
    t = _minkowski(p[:, 0] - p[:, 2])
    u = _minkowski(p[:, 0] - p[:, 3])
    return s, t, u


def test_closed_form_gg_gg():
    p = _events("g g > g g", 64, kin=KIN_C1)
    s, t, u = _mandelstam(p)
    ref = 4.5 * G2 ** 2 * (3 - t * u / s ** 2 - s * u / t ** 2 - s * t / u ** 2)
    np.testing.assert_allclose(oracle_me2("g g > g g", p, ALPHA_S), ref, rtol=1e-13)


def test_closed_form_uubar_gg():
    p = _events("u u~ > g g", 64, kin=KIN_C1)
    s, t, u = _mandelstam(p)
    ref = G2 ** 2 * ((32 / 27) * (t * t + u * u) / (t * u) - (8 / 3) * (t * t + u * u) / s ** 2)
    np.testing.assert_allclose(oracle_me2("u u~ > g g", p, ALPHA_S), ref, rtol=1e-13)


def test_closed_form_uu_uu():
    p = _events("u u > u u", 64, kin=KIN_C1)
    s, t, u = _mandelstam(p)
    ref = G2 ** 2 * ((4 / 9) * ((s * s + u * u) / t ** 2 + (s * s + t * t) / u ** 2) - (8 / 27) * s * s / (t * u))
    np.testing.assert_allclose(oracle_me2("u u > u u", p, ALPHA_S), ref, rtol=1e-13)


def test_closed_form_ug_ug():
    """Crossing of u u~ > g g: ug -> ug = g^4 [-(4/9)(s^2+u^2)/(su) + (s^2+u^2)/t^2]."""
    p = _events("u g > u g", 64, kin=KIN_C1)
    s, t, u = _mandelstam(p)
    ref = G2 ** 2 * (-(4 / 9) * (s * s + u * u) / (s * u) + (s * s + u * u) / t ** 2)
    np.testing.assert_allclose(oracle_me2("u g > u g", p, ALPHA_S), ref, rtol=1e-13)


def test_closed_form_uubar_uubar():
    """Identical-flavour annihilation plus scattering, with the Fermi sign between them."""
    p = _events("u u~ > u u~", 64, kin=KIN_C1)
    s, t, u = _mandelstam(p)
    ref = G2 ** 2 * ((4 / 9) * ((s * s + u * u) / t ** 2 + (u * u + t * t) / s ** 2) - (8 / 27) * u * u / (s * t))
    np.testing.assert_allclose(oracle_me2("u u~ > u u~", p, ALPHA_S), ref, rtol=1e-13)


def test_closed_form_90_degrees():
    """At 90 degrees in the CM frame: 30.375 g^4, ~1.037 g^4 and ~3.26 g^4."""
    e = 250.0
    p = np.array([[[e, 0, 0, e], [e, 0, 0, -e], [e, e, 0, 0], [e, -e, 0, 0]]])
    assert oracle_me2("g g > g g", p, ALPHA_S)[0] / G2 ** 2 == pytest.approx(30.375, rel=1e-13)
    assert oracle_me2("u u~ > g g", p, ALPHA_S)[0] / G2 ** 2 == pytest.approx(28 / 27, rel=1e-13)
    assert oracle_me2("u u > u u", p, ALPHA_S)[0] / G2 ** 2 == pytest.approx(88 / 27, rel=1e-13)


def test_five_gluon_closed_form():
    """Exact for five gluons: (g^6/256) N^3 (N^2-1) 2 sum s_ij^4 sum_{S5/Z5} 1/prod s."""
    p = _events("g g > g g g", 16, seed=3)
    k = p.copy()
    k[:, :2] *= -1.0
    sij = lambda i, j: _minkowski(k[:, i] + k[:, j])
    s4 = sum(sij(i, j) ** 4 for i in range(5) for j in range(i + 1, 5))
    ssum = 0.0
    for perm in itertools.permutations(range(1, 5)):
        w = (0,) + perm
        ssum = ssum + 1.0 / np.prod([sij(w[i], w[(i + 1) % 5]) for i in range(5)], axis=0)
    ref = G2 ** 3 / 256 * 27 * 8 * 2 * s4 * ssum
    np.testing.assert_allclose(oracle_me2("g g > g g g", p, ALPHA_S), ref, rtol=1e-12)


# ------------------------------------------------------------ gauge invariance

@pytest.mark.parametrize("spec,n_ev", [
    ("g g > g g", 8), ("g g > g g g", 4), ("u u~ > g g g", 4), ("u u > u u g", 4),
    ("u u~ > g g g g", 2), ("u u > u u g g", 2), ("g g > g g g g", 1),
])
def test_gauge_invariance(spec, n_ev):
    """Replacing any gluon's polarisation by its momentum must give zero."""
    p = _events(spec, n_ev, seed=5)
    proc = parse_process(spec)
    base = oracle_me2(spec, p, ALPHA_S)
    for leg in range(proc.n):
        if proc.kinds[leg] != "g":
            continue
        # same dimension as the physical case: eps -> k / E
        q = p.copy()
        mg = oracle_me2(spec, q, ALPHA_S, gauge_leg=leg)
        scale = p[:, leg, 0] ** 2
        assert np.max(mg / (base * scale)) < 1e-24


# ------------------------------------------------------------ symmetries

def _boost_rotate(p, rng):
    beta = rng.uniform(-0.7, 0.7, 3)
    b2 = beta @ beta
    gam = 1 / math.sqrt(1 - b2)
    lam = np.eye(4)
    lam[0, 0] = gam
    lam[0, 1:] = lam[1:, 0] = gam * beta
    lam[1:, 1:] += (gam - 1) * np.outer(beta, beta) / b2
    a = rng.normal(size=(3, 3))
    qm, _ = np.linalg.qr(a)
    rot = np.eye(4)
    rot[1:, 1:] = qm
    return p @ (lam @ rot).T


@pytest.mark.parametrize("spec", ["g g > g g g", "u u~ > g g g", "u u > u u g", "u u~ > g g g g"])
def test_lorentz_invariance(spec):
    p = _events(spec, 4, seed=7)
    q = _boost_rotate(p, np.random.default_rng(1))
    np.testing.assert_allclose(oracle_me2(spec, q, ALPHA_S), oracle_me2(spec, p, ALPHA_S), rtol=1e-11)


@pytest.mark.parametrize("spec", ["g g > g g g", "u u~ > g g g", "u u > u u g g"])
def test_scaling(spec):
    p = _events(spec, 4, seed=8)
    n = p.shape[1]
    lam = 3.7
    np.testing.assert_allclose(oracle_me2(spec, lam * p, ALPHA_S),
                               lam ** (8 - 2 * n) * oracle_me2(spec, p, ALPHA_S), rtol=1e-12)


def test_bose_symmetry_final_gluons():
    spec = "g g > g g g"
    p = _events(spec, 4, seed=9)
    base = oracle_me2(spec, p, ALPHA_S)
    for perm in [(2, 4, 3), (4, 3, 2), (3, 2, 4)]:
        q = p[:, [0, 1] + list(perm)]
        np.testing.assert_allclose(oracle_me2(spec, q, ALPHA_S), base, rtol=1e-12)


def test_initial_state_swap_gg():
    spec = "g g > g g g"
    p = _events(spec, 4, seed=10)
    q = p[:, [1, 0, 2, 3, 4]]
    np.testing.assert_allclose(oracle_me2(spec, q, ALPHA_S), oracle_me2(spec, p, ALPHA_S), rtol=1e-12)


@pytest.mark.parametrize("spec", ["u u > u u", "u u > u u g", "u u > u u g g"])
def test_identical_quarks_symmetry(spec):
    """Swapping the two outgoing u quarks, or the two incoming ones."""
    p = _events(spec, 4, seed=11)
    n = p.shape[1]
    base = oracle_me2(spec, p, ALPHA_S)
    out_swap = [0, 1, 3, 2] + list(range(4, n))
    in_swap = [1, 0, 2, 3] + list(range(4, n))
    np.testing.assert_allclose(oracle_me2(spec, p[:, out_swap], ALPHA_S), base, rtol=1e-12)
    np.testing.assert_allclose(oracle_me2(spec, p[:, in_swap], ALPHA_S), base, rtol=1e-12)


def test_fermi_sign_two_lines():
    proc = parse_process("u u > u u")
    signs = sorted(fermion_sign(t, proc) for t, _ in enumerate_diagrams(proc))
    assert signs == [-1, 1]


# ------------------------------------------------------------ helicities

def test_quark_helicity_structural_zeros():
    spec = "u u~ > g g g"
    p = _events(spec, 4, seed=12)
    _, per_hel = oracle_me2(spec, p, ALPHA_S, return_helicities=True)
    hels = helicity_table(5)
    same = hels[:, 0] == hels[:, 1]      # incoming u and u~ with equal helicity
    assert np.all(per_hel[same] == 0.0)
    assert np.all(per_hel[~same].max(axis=0) > 0)


def test_all_gluon_helicity_zeros():
    """All-plus and single-minus (all-outgoing labels) amplitudes vanish."""
    spec = "g g > g g g g"
    p = _events(spec, 2, seed=13)
    _, per_hel = oracle_me2(spec, p, ALPHA_S, return_helicities=True)
    hels = helicity_table(6).copy()
    hels[:, :2] *= -1                   # incoming legs flip in all-outgoing labels
    nminus = (hels < 0).sum(axis=1)
    small = (nminus <= 1) | (nminus >= 5)
    assert per_hel[small].max() < 1e-20 * per_hel.max()
    assert per_hel[~small].min() > 0


@pytest.mark.parametrize("spec", ["g g > g g g", "u u~ > g g g", "u u > u u g", "g g > g g g g"])
def test_helicity_flip_symmetry(spec):
    """Flipping every helicity leaves the colour-summed |M_lambda|^2 unchanged."""
    p = _events(spec, 2, seed=14)
    _, per_hel = oracle_me2(spec, p, ALPHA_S, return_helicities=True)
    n = p.shape[1]
    flip = (np.arange(1 << n) ^ ((1 << n) - 1))
    np.testing.assert_allclose(per_hel[flip], per_hel, rtol=1e-11, atol=1e-13 * per_hel.max())


def test_parke_taylor_mhv():
    spec = "g g > g g g g"
    p = _events(spec, 3, seed=15)
    k = p.copy()
    k[:, :2] *= -1
    sij = lambda i, j: _minkowski(k[:, i] + k[:, j])
    jamp, hels = oracle_amplitudes(spec, p, ALPHA_S)
    basis = colour_basis(parse_process(spec))
    out_hel = hels.copy()
    out_hel[:, :2] *= -1
    ratios = []
    for h in range(hels.shape[0]):
        neg = np.nonzero(out_hel[h] < 0)[0]
        if len(neg) != 2:
            continue
        i, j = neg
        for a, desc in enumerate(basis):
            w = desc[0][2]
            ps = np.prod([np.abs(sij(w[x], w[(x + 1) % 6])) for x in range(6)], axis=0)
            ratios.append(np.abs(jamp[h, :, a]) ** 2 * ps / sij(i, j) ** 4)
    ratios = np.array(ratios)
    assert np.max(np.abs(ratios / ratios[0] - 1)) < 1e-11


@pytest.mark.parametrize("spec,n_ev", [("g g > g g", 4), ("g g > g g g", 3), ("g g > g g g g", 2)])
def test_berends_giele_matches_jamps(spec, n_ev):
    """Trace-basis amplitudes equal colour-ordered Berends-Giele amplitudes x one constant."""
    p = _events(spec, n_ev, seed=16)
    proc = parse_process(spec)
    jamp, hels = oracle_amplitudes(spec, p, ALPHA_S)
    bg = bg_amplitudes(spec, p, hels)
    basis = colour_basis(proc)
    g = math.sqrt(G2)
    n = proc.n
    ratios = []
    for a, desc in enumerate(basis):
        a_bg = bg[trace_word_to_bg(desc[0][2], proc.root)]
        mask = np.abs(a_bg) > 1e-9 * np.abs(a_bg).max()
        ratios.append((jamp[..., a][mask] / a_bg[mask]))
    r = np.concatenate(ratios)
    assert np.max(np.abs(r / r[0] - 1)) < 1e-10
    # magnitude fixed by the normalisations: J = 2^{n/2} g^{n-2} A
    assert abs(abs(r[0]) / (2 ** (n / 2) * g ** (n - 2)) - 1) < 1e-12


@pytest.mark.parametrize("spec,n_ev", [("u u~ > g g", 4), ("u u~ > g g g", 3), ("u u~ > g g g g", 2),
                                       ("u g > u g g", 3), ("g u~ > g g u~", 2)])
def test_berends_giele_quark_line_matches_jamps(spec, n_ev):
    """Chain-basis amplitudes of one quark line equal the colour-ordered Berends-Giele quark-line
    recursion times one real positive constant, 2^{k/2} g^{n-2} for k gluons (t = T / sqrt2 per
    generator of the chain, one g per vertex)."""
    p = _events(spec, n_ev, seed=16)
    proc = parse_process(spec)
    jamp, hels = oracle_amplitudes(spec, p, ALPHA_S)
    _, bg = bg_quark_amplitudes(spec, p, hels)
    basis = colour_basis(proc)
    scale = 0.0
    ratios = []
    for a, desc in enumerate(basis):
        a_bg = bg[tuple(desc[0][2])]
        scale = max(scale, np.abs(a_bg).max())
    for a, desc in enumerate(basis):
        a_bg = bg[tuple(desc[0][2])]
        big = np.abs(a_bg) > 1e-9 * scale
        # where the recursion vanishes (helicity zeros) the diagram sum vanishes too
        assert np.all(np.abs(jamp[..., a][~big]) < 1e-9 * np.abs(jamp).max())
        ratios.append(jamp[..., a][big] / a_bg[big])
    r = np.concatenate(ratios)
    k = sum(1 for x in proc.kinds if x == "g")
    expected = 2 ** (k / 2) * math.sqrt(G2) ** (proc.n - 2)
    assert np.max(np.abs(r / expected - 1)) < 1e-10


def test_parke_taylor_quark_line():
    """One quark line, MHV: in the all-outgoing convention, with f- / f+ the quark-line ends of
    negative / positive helicity and i the one negative-helicity gluon, every colour-ordered
    |A(sigma)|^2 is |s_{f- i}|^3 |s_{f+ i}| / prod_cyclic |s_{adjacent}| times one constant (the
    cyclic order runs from the row end of the chain over the gluons to its column end)."""
    spec = "u u~ > g g g g"
    p = _events(spec, 3, seed=19)
    proc = parse_process(spec)
    k = p.copy()
    k[:, :2] *= -1                                   # all momenta outgoing
    sij = lambda i, j: np.abs(_minkowski(k[:, i] + k[:, j]))
    jamp, hels = oracle_amplitudes(spec, p, ALPHA_S)
    out_hel = hels.copy()
    out_hel[:, :2] *= -1                             # incoming helicity h is outgoing -h
    basis = colour_basis(proc)
    row, col = basis[0][0][0], basis[0][0][1]
    gl = [i for i, x in enumerate(proc.kinds) if x == "g"]
    ratios, seen = [], 0
    for h in range(hels.shape[0]):
        neg_g = [i for i in gl if out_hel[h, i] < 0]
        if len(neg_g) != 1 or out_hel[h, row] == out_hel[h, col]:
            continue
        i = neg_g[0]
        fm, fp = (row, col) if out_hel[h, row] < 0 else (col, row)
        seen += 1
        for a, desc in enumerate(basis):
            order = [row] + list(desc[0][2]) + [col]
            ps = np.prod([sij(order[x], order[(x + 1) % len(order)]) for x in range(len(order))], axis=0)
            ratios.append(np.abs(jamp[h, :, a]) ** 2 * ps / (sij(fm, i) ** 3 * sij(fp, i)))
    ratios = np.array(ratios)
    assert seen == 8                                   # 2 quark-helicity assignments x 4 gluons
    assert np.max(np.abs(ratios / ratios[0] - 1)) < 1e-10


# ------------------------------------------------------------ exhaustive colour

@pytest.mark.parametrize("spec", ["g g > g g", "u u~ > g g", "u u > u u", "u u~ > g g g",
                                  "u u > u u g", "g g > g g g"])
def test_exhaustive_colour_sum(spec):
    """sum over every explicit colour assignment of |sum_d C_d(c) A_d|^2, no basis at all."""
    p = _events(spec, 3, seed=17)
    cd = colour_data(spec)
    proc = cd.proc
    hels = helicity_table(proc.n)
    waves, moms = _externals(proc, p, hels, None)
    g = math.sqrt(G2)
    amps = np.stack([cd.signs[d] * _evaluate(t, rk, proc, waves, moms, g)
                     for d, (t, rk) in enumerate(cd.diagrams)])          # [D, H, N]
    c = all_assignments(proc)
    cvals = np.stack([diagram_colour_values(t, rk, proc, c) for t, rk in cd.diagrams], axis=1)  # [m, D]
    m_c = np.einsum("md,dhn->mhn", cvals, amps)
    ref = (np.abs(m_c) ** 2).sum(axis=(0, 1)) / (4 * proc.initial_colour_dof())
    np.testing.assert_allclose(oracle_me2(spec, p, ALPHA_S), ref, rtol=1e-12)


# ------------------------------------------------------------ wavefunctions

def _momenta(rng, n=32):
    v = rng.normal(size=(n, 3)) * 100
    v[0] = [0, 0, 70.0]      # beam axis +z
    v[1] = [0, 0, -45.0]     # beam axis -z
    e = np.linalg.norm(v, axis=1)
    return np.concatenate([e[:, None], v], axis=1)


def test_spinors_dirac_equation_and_current():
    p = _momenta(np.random.default_rng(2))
    ps = L.slash(p)
    for lam in (-1, 1):
        for sp in (L.spinor_u(p, lam), L.spinor_v(p, lam)):
            assert np.abs(np.einsum("nij,nj->ni", ps, sp)).max() < 1e-10
            cur = np.einsum("ni,mij,nj->nm", L.dirac_bar(sp), L.GAMMA, sp)
            np.testing.assert_allclose(cur.real, 2 * p, atol=1e-9)
            assert np.abs(cur.imag).max() < 1e-9
    # helicity: u(+) is right-handed (lower two components in the chiral basis)
    assert np.abs(L.spinor_u(p, 1)[:, :2]).max() == 0
    assert np.abs(L.spinor_u(p, -1)[:, 2:]).max() == 0


def test_polarisations():
    p = _momenta(np.random.default_rng(3))
    ep, em = L.polarisation(p, 1), L.polarisation(p, -1)
    for e in (ep, em):
        assert np.abs(L.mdot(e, p)).max() < 1e-9
        np.testing.assert_allclose(L.mdot(e, e.conj()), -1.0, atol=1e-12)
    assert np.abs(L.mdot(ep, em.conj())).max() < 1e-12
    comp = np.einsum("ni,nj->nij", ep[:, 1:], ep[:, 1:].conj()) + np.einsum("ni,nj->nij", em[:, 1:], em[:, 1:].conj())
    khat = p[:, 1:] / p[:, :1]
    np.testing.assert_allclose(comp, np.eye(3)[None] - np.einsum("ni,nj->nij", khat, khat), atol=1e-12)
    # helicity +1 along +z is -(0, 1, i, 0)/sqrt2
    np.testing.assert_allclose(ep[0], np.array([0, -1, -1j, 0]) / np.sqrt(2), atol=1e-15)


# ------------------------------------------------------------ seven gluons
# The literal colour sum over 8^7 assignments and 720 basis elements is out of reach of the
# diagram oracle, so g g > g g g g g is computed by the Berends-Giele route with the trace
# colour matrix built from one trace tensor; these pins fix that route.

@pytest.mark.parametrize("spec", ["g g > g g", "g g > g g g", "g g > g g g g"])
def test_berends_giele_me2_equals_diagram_oracle(spec):
    from oracle.berends_giele import bg_me2
    p = _events(spec, 4, seed=23)
    np.testing.assert_allclose(bg_me2(spec, p, ALPHA_S), oracle_me2(spec, p, ALPHA_S), rtol=1e-12)


@pytest.mark.parametrize("n", [4, 5])
def test_trace_colour_matrix_equals_literal_colour_sum(n):
    """The permuted-tensor construction equals the oracle's sum over every colour assignment."""
    from oracle.berends_giele import trace_colour_matrix
    spec = "g g > " + " ".join(["g"] * (n - 2))
    words, nmat = trace_colour_matrix(n)
    cd = colour_data(spec)
    basis = colour_basis(cd.proc)
    order = [words.index(trace_word_to_bg(desc[0][2], cd.proc.root)) for desc in basis]
    np.testing.assert_allclose(nmat.real[np.ix_(order, order)], cd.N, rtol=0, atol=1e-15)
    assert np.abs(nmat.imag).max() < 1e-15


def test_seven_gluon_colour_matrix_table3():
    """Table 3: 45 distinct non-zero colour-matrix values for g g > g g g g g."""
    from oracle.berends_giele import trace_colour_matrix
    from oracle.colour import _rationalise
    want = {r[0]: int(r[1]) for r in _table("paper_table3.txt")}["g g > g g g g g"]
    words, nmat = trace_colour_matrix(7)
    assert len(words) == 720
    n = nmat.real
    assert np.abs(nmat.imag).max() < 1e-14 and np.allclose(n, n.T, rtol=0, atol=1e-15)
    vals = {_rationalise(x) for i in range(720) for x in n[i, i:] if abs(x) > 1e-13}
    assert len(vals) == want
    assert np.linalg.eigvalsh(n).min() > -1e-12


def test_seven_gluon_parke_taylor_and_symmetries():
    """Berends-Giele for 7 gluons: MHV partial amplitudes follow Parke-Taylor, all-plus and
    one-minus vanish, and |M|^2 is symmetric under exchange of final gluons."""
    from oracle.berends_giele import bg_me2
    spec = "g g > g g g g g"
    p = _events(spec, 2, seed=29)
    k = p.copy()
    k[:, :2] *= -1
    sij = lambda i, j: _minkowski(k[:, i] + k[:, j])
    hels = helicity_table(7)
    amps = bg_amplitudes(spec, p, hels)
    out_hel = hels.copy()
    out_hel[:, :2] *= -1
    ratios, zeros, scale = [], [], 0.0
    for word, a in list(amps.items())[::37]:
        cyc = list(word) + [6]
        ps = np.prod([np.abs(sij(cyc[x], cyc[(x + 1) % 7])) for x in range(7)], axis=0)
        for h in range(hels.shape[0]):
            neg = np.nonzero(out_hel[h] < 0)[0]
            scale = max(scale, np.abs(a[h]).max())
            if len(neg) == 2:
                i, j = neg
                ratios.append(np.abs(a[h]) ** 2 * ps / sij(i, j) ** 4)
            elif len(neg) <= 1 or len(neg) >= 6:
                zeros.append(np.abs(a[h]).max())
    ratios = np.array(ratios)
    assert np.max(np.abs(ratios / ratios[0] - 1)) < 1e-10
    assert max(zeros) < 1e-12 * scale
    m = bg_me2(spec, p, ALPHA_S)
    swapped = p[:, [0, 1, 4, 2, 6, 3, 5]]
    np.testing.assert_allclose(bg_me2(spec, swapped, ALPHA_S), m, rtol=1e-12)
