"""Pins of the phase-space / cuts / cross-section oracle against closed forms and an
independent implementation (no GPU).

* massless phase-space volume: Phi_2 = 1/(8 pi), Phi_3 = s / (256 pi^3) (textbook values);
* oracle RAMBO (event-by-event) against the vectorised input generator on the same uniforms;
* momentum conservation and masslessness; flat 3-body Dalitz density (E[x^2] = 1/2);
* cuts on hand-built events either side of each threshold;
* the Monte Carlo cross section of g g > g g and u g > u g at fixed sqrt(s) against a
  one-dimensional quadrature of their closed-form |M|^2 (checks flux, phase-space weight,
  identical-particle factor and units at once).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle_me2
from oracle import phase_space as ops
from phasespace import KIN_C1, KIN_C2, rambo_massless, rambo_uniforms

ALPHA_S = 0.118
G2 = 4 * math.pi * ALPHA_S


def test_phase_space_volume_closed_forms():
    for s in (1.0, 2.5e5, 4e6):
        assert ops.phase_space_volume(2, s) == pytest.approx(1 / (8 * math.pi), rel=1e-15)
        assert ops.phase_space_volume(3, s) == pytest.approx(s / (256 * math.pi ** 3), rel=1e-14)


class _Fixed:
    def __init__(self, u):
        self.u = u

    def random(self, shape):
        assert shape == self.u.shape
        return self.u


@pytest.mark.parametrize("nf", [2, 3, 4, 5, 7])
def test_rambo_matches_vectorised_generator(nf):
    rs, u = rambo_uniforms(300, nf, KIN_C2, seed=3)
    mom, w = ops.rambo(rs, u)
    ref = rambo_massless(_Fixed(u), nf, rs)
    np.testing.assert_allclose(mom[:, 2:], ref, rtol=0, atol=1e-12 * rs.max())
    assert np.all(w == np.array([ops.phase_space_volume(nf, r * r) for r in rs]))


@pytest.mark.parametrize("nf", [2, 3, 6])
def test_rambo_conservation_and_mass_shell(nf):
    rs, u = rambo_uniforms(500, nf, KIN_C2, seed=5)
    mom, _ = ops.rambo(rs, u)
    tot = mom[:, 2:].sum(axis=1)
    np.testing.assert_allclose(tot[:, 0], rs, rtol=1e-13)
    assert np.abs(tot[:, 1:]).max() <= 1e-12 * rs.max()
    m2 = mom[..., 0] ** 2 - (mom[..., 1:] ** 2).sum(axis=-1)
    assert np.abs(m2).max() <= 1e-11 * rs.max() ** 2
    np.testing.assert_array_equal(mom[:, 0], np.stack([rs / 2, 0 * rs, 0 * rs, rs / 2], 1))


def test_rambo_three_body_dalitz_is_flat():
    """Massless 3-body phase space is flat in (E1, E2): x = 2E1/sqrt(s) has density 2x on [0, 1]."""
    rs, u = rambo_uniforms(40000, 3, KIN_C1, seed=9)
    mom, _ = ops.rambo(rs, u)
    x = 2 * mom[:, 2, 0] / rs
    assert abs(np.mean(x) - 2 / 3) < 0.006
    assert abs(np.mean(x * x) - 0.5) < 0.006
    assert abs(np.mean(mom[:, 2, 3] / mom[:, 2, 0])) < 0.02       # isotropic: <cos theta> = 0


def _parton(pt, eta, phi):
    return [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]


def test_cuts_either_side_of_each_threshold():
    ok = [_parton(50, 0.3, 0.0), _parton(60, -1.0, 2.0)]
    assert ops.passes_cuts(ok, 20, 2.5, 0.4)
    assert not ops.passes_cuts([_parton(19.9, 0.3, 0.0), ok[1]], 20, 2.5, 0.4)
    assert ops.passes_cuts([_parton(20.1, 0.3, 0.0), ok[1]], 20, 2.5, 0.4)
    assert not ops.passes_cuts([_parton(50, 2.51, 0.0), ok[1]], 20, 2.5, 0.4)
    assert not ops.passes_cuts([_parton(50, -2.51, 0.0), ok[1]], 20, 2.5, 0.4)
    assert ops.passes_cuts([_parton(50, 2.49, 0.0), ok[1]], 20, 2.5, 0.4)
    close = [_parton(50, 0.3, 0.0), _parton(40, 0.3 + 0.2, 0.3)]      # dR = 0.3606
    assert not ops.passes_cuts(close, 20, 2.5, 0.4)
    assert ops.passes_cuts(close, 20, 2.5, 0.0)                        # pair cut off
    wrap = [_parton(50, 0.0, 3.1), _parton(40, 0.0, -3.1)]             # dphi wraps to 0.083
    assert not ops.passes_cuts(wrap, 20, 2.5, 0.4)
    assert ops.cut_margin(close, 20, 2.5, 0.4) == pytest.approx((0.4 - math.hypot(0.2, 0.3)) / 0.4, rel=1e-9)


def test_final_state_symmetry():
    assert ops.final_state_symmetry("g g > g g g g") == 24
    assert ops.final_state_symmetry("u u > u u g g") == 4
    assert ops.final_state_symmetry("u u~ > g g g") == 6
    assert ops.final_state_symmetry("u g > u g") == 1


@pytest.mark.parametrize("spec", ["g g > g g", "u g > u g"])
def test_cross_section_matches_quadrature(spec):
    rs = 500.0
    s = rs * rs
    c_max = math.tanh(2.5)          # the eta cut binds: pT > 20 GeV only needs |cos| < 0.9968

    def me2_closed(c):
        t, u = -s * (1 - c) / 2, -s * (1 + c) / 2
        if spec == "g g > g g":
            return 4.5 * G2 ** 2 * (3 - t * u / s ** 2 - s * u / t ** 2 - s * t / u ** 2)
        return G2 ** 2 * (-(4 / 9) * (s * s + u * u) / (s * u) + (s * s + u * u) / t ** 2)

    sym = 2 if spec == "g g > g g" else 1
    quad = integrate.quad(me2_closed, -c_max, c_max, epsabs=0, epsrel=1e-11)[0]
    exact = ops.GEV2_PB * quad / (16 * math.pi) / (2 * s * sym)
    n = 50000
    _, u = rambo_uniforms(n, 2, KIN_C1, seed=21)
    mean, err, f = ops.cross_section(spec, np.full(n, rs), u, lambda p: oracle_me2(spec, p, ALPHA_S),
                                     20.0, 2.5, 0.0)
    assert err < 0.04 * mean
    assert abs(mean - exact) < 4 * err, (mean, exact, err)
    assert np.count_nonzero(f) < n                     # some events fail the cuts
