"""Oracle for the device phase space, jet cuts and event weights (test infrastructure only).

Event by event, in plain Python floats (float64), following:

* massless RAMBO, Kleiss, Stirling and Ellis, Comput. Phys. Commun. 40 (1986) 359:
  for each of the n final partons take a direction uniform on the sphere
  (cos theta = 2 u0 - 1, phi = 2 pi u1) and an energy q0 = -log(u2 u3) (density
  q0 exp(-q0)); with Q the sum of these massless vectors and M its mass, boost
  every vector by the Lorentz transformation that takes Q to rest
  (b = -Q/M, gamma = Q0/M, a = 1/(1+gamma)) and scale by x = sqrt(s)/M.  The weight
  is the same for every event: the volume of massless n-body phase space,
  (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!);
* the jet cuts of the paper's section 2.2 (eqs. cuts) with Delta R in place of the
  relative-pT cut: pT > pT_min, |eta| < eta_max, Delta R_ij > Delta R_min, strict;
* the partonic cross section of the paper's eq. (cross-section) at fixed sqrt(s)
  (no parton densities): sigma-hat = 1/(2 s) 1/S integral dPhi_n |M|^2 Theta(cuts),
  S = product of factorials of identical final partons, in pb.
"""
from __future__ import annotations

import math

import numpy as np

GEV2_PB = 0.3893793721e9   # (hbar c)^2 in pb GeV^2


def phase_space_volume(n: int, s: float) -> float:
    """Volume of massless n-body phase space at invariant mass squared s."""
    return ((2.0 * math.pi) ** (4 - 3 * n) * (math.pi / 2.0) ** (n - 1) * s ** (n - 2)
            / (math.factorial(n - 1) * math.factorial(n - 2)))


def rambo_event(sqrt_s: float, u) -> tuple:
    """One event: uniforms u[n][4] -> (momenta [n+2][4] incl. beams, weight)."""
    n = len(u)
    q = []
    for ui in u:
        c = 2.0 * ui[0] - 1.0
        st = math.sqrt(max(0.0, 1.0 - c * c))
        phi = 2.0 * math.pi * ui[1]
        e = -math.log(ui[2] * ui[3])
        q.append([e, e * st * math.cos(phi), e * st * math.sin(phi), e * c])
    big = [sum(v[k] for v in q) for k in range(4)]
    m = math.sqrt(big[0] ** 2 - big[1] ** 2 - big[2] ** 2 - big[3] ** 2)
    b = [-big[k] / m for k in (1, 2, 3)]
    gamma = big[0] / m
    a = 1.0 / (1.0 + gamma)
    x = sqrt_s / m
    out = [[sqrt_s / 2, 0.0, 0.0, sqrt_s / 2], [sqrt_s / 2, 0.0, 0.0, -sqrt_s / 2]]
    for v in q:
        bq = b[0] * v[1] + b[1] * v[2] + b[2] * v[3]
        out.append([x * (gamma * v[0] + bq)] + [x * (v[1 + k] + b[k] * v[0] + a * bq * b[k]) for k in range(3)])
    return np.array(out), phase_space_volume(n, sqrt_s * sqrt_s)


def rambo(sqrt_s, uniforms) -> tuple:
    """All events: (momenta [N][n+2][4], weights [N])."""
    moms, ws = [], []
    for rs, u in zip(np.asarray(sqrt_s, dtype=float), np.asarray(uniforms, dtype=float)):
        p, w = rambo_event(float(rs), u)
        moms.append(p)
        ws.append(w)
    n = np.asarray(uniforms).shape[1] if len(moms) == 0 else moms[0].shape[0] - 2
    return (np.array(moms).reshape(-1, n + 2, 4), np.array(ws))


def rambo_gamma(uniforms) -> np.ndarray:
    """Per event the Lorentz factor Q0/M of RAMBO's boost.  Rounding differences in the isotropic
    vectors reach the boosted momenta amplified by up to gamma^2 (nearly collinear draws), which
    sets how closely two correct implementations can agree."""
    out = []
    for u in np.asarray(uniforms, dtype=float):
        big = [0.0, 0.0, 0.0, 0.0]
        for ui in u:
            c = 2.0 * ui[0] - 1.0
            st = math.sqrt(max(0.0, 1.0 - c * c))
            phi = 2.0 * math.pi * ui[1]
            e = -math.log(ui[2] * ui[3])
            for k, v in enumerate((e, e * st * math.cos(phi), e * st * math.sin(phi), e * c)):
                big[k] += v
        out.append(big[0] / math.sqrt(big[0] ** 2 - big[1] ** 2 - big[2] ** 2 - big[3] ** 2))
    return np.array(out)


def _pt_eta_phi(p):
    pt = math.hypot(p[1], p[2])
    pa = math.sqrt(pt * pt + p[3] * p[3])
    eta = 0.5 * math.log((pa + p[3]) / (pa - p[3]))
    return pt, eta, math.atan2(p[2], p[1])


def passes_cuts(finals, pt_min: float, eta_max: float, dr_min: float) -> bool:
    """Every final parton hard and central enough, every pair separated (dr_min <= 0: no pair cut)."""
    kin = []
    for p in finals:
        pt, eta, phi = _pt_eta_phi(p)
        if not (pt > pt_min and abs(eta) < eta_max):
            return False
        kin.append((eta, phi))
    if dr_min > 0:
        for i in range(len(kin)):
            for j in range(i + 1, len(kin)):
                dphi = abs(kin[i][1] - kin[j][1])
                if dphi > math.pi:
                    dphi = 2.0 * math.pi - dphi
                if not (math.hypot(kin[i][0] - kin[j][0], dphi) > dr_min):
                    return False
    return True


def cut_margin(finals, pt_min: float, eta_max: float, dr_min: float) -> float:
    """Smallest relative distance of any cut variable from its threshold (for tie handling in tests)."""
    out = math.inf
    kin = []
    for p in finals:
        pt, eta, phi = _pt_eta_phi(p)
        out = min(out, abs(pt - pt_min) / pt_min if pt_min > 0 else math.inf, abs(abs(eta) - eta_max) / eta_max)
        kin.append((eta, phi))
    if dr_min > 0:
        for i in range(len(kin)):
            for j in range(i + 1, len(kin)):
                dphi = abs(kin[i][1] - kin[j][1])
                if dphi > math.pi:
                    dphi = 2.0 * math.pi - dphi
                out = min(out, abs(math.hypot(kin[i][0] - kin[j][0], dphi) - dr_min) / dr_min)
    return out


def final_state_symmetry(spec: str) -> int:
    """Product of factorials of the multiplicities of identical final partons."""
    finals = spec.split(">")[1].split()
    out = 1
    for name in set(finals):
        out *= math.factorial(finals.count(name))
    return out


def event_weights(spec: str, momenta, me2, pt_min: float, eta_max: float, dr_min: float):
    """f_e = (hbar c)^2 Phi_n(s) |M|^2 Theta(cuts) / (2 s S) in pb, per event."""
    sym = final_state_symmetry(spec)
    out = []
    for p, m in zip(np.asarray(momenta), np.asarray(me2)):
        s = (p[0][0] + p[1][0]) ** 2 - sum((p[0][k] + p[1][k]) ** 2 for k in (1, 2, 3))
        n = p.shape[0] - 2
        ok = passes_cuts(p[2:], pt_min, eta_max, dr_min)
        out.append(GEV2_PB * phase_space_volume(n, s) * m / (2.0 * s * sym) if ok else 0.0)
    return np.array(out)


def cross_section(spec: str, sqrt_s, uniforms, me2_fn, pt_min: float, eta_max: float, dr_min: float):
    """Monte Carlo estimate (mean, standard error) of sigma-hat in pb and the event weights.

    me2_fn(momenta [N][n+2][4]) -> |M|^2 [N]; for the QCD processes this is the
    oracle's oracle_me2 with the coupling bound in."""
    mom, _ = rambo(sqrt_s, uniforms)
    f = event_weights(spec, mom, me2_fn(mom), pt_min, eta_max, dr_min)
    n = len(f)
    mean = float(np.mean(f))
    err = float(np.std(f, ddof=1) / math.sqrt(n)) if n > 1 else math.inf
    return mean, err, f
