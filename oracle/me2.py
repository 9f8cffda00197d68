"""Colour- and helicity-summed |M|^2 from independent Feynman diagrams (oracle).

Follows the paper's section 2.1 in order:
  eq. matrix-element           the amplitude is the sum over all diagrams;
  eq. color-amplitude          J_alpha = sum_d c_{d alpha} A_d per helicity;
  eq. color-matrix             N from the literal colour sum (colour module);
  eq. color-averaged-amplitude sum_{alpha beta} J_alpha N_{alpha beta} J_beta^*;
  helicity sum-average         1/2 * 1/2 * sum over all helicity configurations.

Helicity configuration h (0 <= h < 2^n) gives leg i the helicity +1 when bit i
of h is set and -1 otherwise (physical helicities of the particles as they
appear in the process string).

The output is not multiplied by the identical-particle factor, which belongs
to the phase space (section 2.1, remark after eq. phase-space).
"""
from __future__ import annotations

import math

import numpy as np

from . import lorentz as L
from .colour import colour_data


def helicity_table(n: int) -> np.ndarray:
    h = np.arange(1 << n)
    return np.where((h[:, None] >> np.arange(n)[None, :]) & 1, 1, -1)


def _externals(proc, p, hels, gauge_leg):
    """Wavefunctions [H, N, 4] and vertex-incoming momenta [N, 4] per leg."""
    waves, moms = [], []
    for i in range(proc.n):
        pi = p[:, i, :]
        both = {}
        for lam in (-1, 1):
            kind = proc.kinds[i]
            if kind == "g":
                w = L.polarisation(pi, lam)
                if not proc.incoming[i]:
                    w = w.conj()
            elif kind == "qi":
                w = L.spinor_u(pi, lam) if proc.flavours[i] == "u" else L.spinor_v(pi, lam)
            else:
                w = L.spinor_u(pi, lam) if proc.flavours[i] == "u" else L.spinor_v(pi, lam)
                w = L.dirac_bar(w)
            if gauge_leg == i:
                w = pi.astype(np.complex128)
            both[lam] = w
        waves.append(np.where((hels[:, i] > 0)[:, None, None], both[1][None], both[-1][None]))
        moms.append(pi if proc.incoming[i] else -pi)
    return waves, moms


def _evaluate(tree, root_kind, proc, waves, moms, g):
    def ev(t, prop=True):
        tag = t[0]
        if tag == "leg":
            return waves[t[1]], moms[t[1]]
        if tag == "ggg":
            (ja, ka), (jb, kb) = ev(t[1]), ev(t[2])
            v, k = L.v_ggg(ja, ka, jb, kb, g), ka + kb
            return (L.prop_gluon(v, k) if prop else v), k
        if tag == "gggg":
            (ja, ka), (jb, kb), (jc, kc) = ev(t[2]), ev(t[3]), ev(t[4])
            v, k = L.v_gggg(t[1], ja, jb, jc, g), ka + kb + kc
            return (L.prop_gluon(v, k) if prop else v), k
        if tag == "qqg_i":
            (f, kf), (ja, ka) = ev(t[1]), ev(t[2])
            v, k = L.v_qqg_col(f, ja, g), kf + ka
            return (L.prop_quark_col(v, k) if prop else v), k
        if tag == "qqg_o":
            (gb, kg), (ja, ka) = ev(t[1]), ev(t[2])
            v, k = L.v_qqg_row(gb, ja, g), kg + ka
            return (L.prop_quark_row(v, -k) if prop else v), k
        if tag == "qq_g":
            (f, kf), (gb, kg) = ev(t[1]), ev(t[2])
            v, k = L.v_qq_g(f, gb, g), kf + kg
            return (L.prop_gluon(v, k) if prop else v), k
        raise AssertionError(tag)

    v, _ = ev(tree, prop=False)
    w = waves[proc.root]
    if root_kind == "g":
        return L.mdot(v, w)
    return np.einsum("...i,...i->...", v, w)


def oracle_amplitudes(spec: str, momenta: np.ndarray, alpha_s: float, hels=None, gauge_leg=None):
    """Colour-basis amplitudes J [H, N, K] and the helicity table [H, n]."""
    cd = colour_data(spec)
    proc = cd.proc
    p = np.asarray(momenta, dtype=np.float64)
    assert p.ndim == 3 and p.shape[1:] == (proc.n, 4), p.shape
    if hels is None:
        hels = helicity_table(proc.n)
    g = math.sqrt(4.0 * math.pi * alpha_s)
    waves, moms = _externals(proc, p, hels, gauge_leg)
    jamp = np.zeros((hels.shape[0], p.shape[0], cd.n_colours), dtype=np.complex128)
    for d, (tree, rk) in enumerate(cd.diagrams):
        amp = cd.signs[d] * _evaluate(tree, rk, proc, waves, moms, g)
        nz = np.nonzero(np.abs(cd.coef[d]) > 1e-12)[0]
        jamp[..., nz] += amp[..., None] * cd.coef[d, nz]
    return jamp, hels


def colour_sum(jamp: np.ndarray, nmat: np.ndarray) -> np.ndarray:
    """sum_{alpha beta} J_alpha N_{alpha beta} J_beta^* (real part), [H, N]."""
    return np.einsum("...a,ab,...b->...", jamp, nmat, jamp.conj()).real


def oracle_me2(spec: str, momenta: np.ndarray, alpha_s: float, gauge_leg=None,
               return_helicities: bool = False, chunk: int = 64):
    """Spin/colour averaged |M|^2 for every event: float64 [N].

    momenta: float64 [N][n][4] (E, px, py, pz), physical in/out momenta in the
    order of the process string.  With return_helicities=True also returns the
    per-helicity colour sums [H, N] (before the 1/4 average).
    """
    cd = colour_data(spec)
    p = np.asarray(momenta, dtype=np.float64)
    outs, hel_outs = [], []
    for lo in range(0, p.shape[0], chunk):
        jamp, _ = oracle_amplitudes(spec, p[lo:lo + chunk], alpha_s, gauge_leg=gauge_leg)
        per_hel = colour_sum(jamp, cd.N)
        outs.append(0.25 * per_hel.sum(axis=0))
        hel_outs.append(per_hel)
    me2 = np.concatenate(outs) if outs else np.zeros(0)
    if return_helicities:
        return me2, (np.concatenate(hel_outs, axis=1) if hel_outs else np.zeros((0, 0)))
    return me2
