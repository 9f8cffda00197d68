"""RAMBO massless phase-space generator with reject-and-resample jet cuts.

Momenta follow Kleiss, Stirling and Ellis, Comput. Phys. Commun. 40 (1986) 359
(RAMBO): n isotropic massless vectors with energies drawn from q0*exp(-q0) are
boosted and scaled so that they sum to (sqrt(s), 0, 0, 0).

The partonic collision is taken in its centre-of-mass frame, which is also the
lab frame here because no parton densities are folded in (the paper's
section 2.1 convolution is out of scope).  Incoming partons move along +z and
-z with energy sqrt(s)/2 each.

Cuts are those of the paper's section 2.2 (eqs. cuts): |eta| < 2.5 and
pT > 20 GeV on every final-state parton, optionally Delta R_ij > 0.4 between
every pair (this replaces the paper's relative-pT cut pT_ij).  An event that
fails any cut is discarded whole and drawn again.

Layout of the returned array: float64 [N][n_ext][4] with components
(E, px, py, pz); particle order is a, b, then the finals.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Kinematics:
    """How the partonic energy and the cuts of one workload are chosen."""

    sqrt_s_min: float          # GeV; equal to sqrt_s_max for fixed energy
    sqrt_s_max: float
    pt_min: float = 20.0       # GeV, eq. (cuts-pt)
    eta_max: float = 2.5       # eq. (cuts-eta)
    delta_r_min: float | None = None  # pairwise Delta R cut, None = off


# gg -> gg reference workload: fixed sqrt(s) = 500 GeV, pT and eta cuts only.
KIN_C1 = Kinematics(500.0, 500.0)
# Multi-jet workloads: sqrt(s) uniform in [300, 2000] GeV plus Delta R > 0.4.
KIN_C2 = Kinematics(300.0, 2000.0, delta_r_min=0.4)
# Serving workload: sqrt(s) uniform in [300, 3000] GeV plus Delta R > 0.4.
KIN_C5 = Kinematics(300.0, 3000.0, delta_r_min=0.4)


def rambo_massless(rng: np.random.Generator, n_final: int, sqrt_s: np.ndarray) -> np.ndarray:
    """Draw len(sqrt_s) events of n_final massless momenta summing to (sqrt_s, 0).

    Returns float64 [N][n_final][4] (E, px, py, pz).
    """
    sqrt_s = np.asarray(sqrt_s, dtype=np.float64)
    n = sqrt_s.shape[0]
    r = rng.random((n, n_final, 4))
    # isotropic massless vectors, energy density q0 * exp(-q0)
    cos_t = 2.0 * r[..., 0] - 1.0
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = 2.0 * math.pi * r[..., 1]
    q0 = -np.log(r[..., 2] * r[..., 3] + 1e-300)
    q = np.empty((n, n_final, 4))
    q[..., 0] = q0
    q[..., 1] = q0 * sin_t * np.cos(phi)
    q[..., 2] = q0 * sin_t * np.sin(phi)
    q[..., 3] = q0 * cos_t
    big_q = q.sum(axis=1)                                  # [N,4]
    mass = np.sqrt(big_q[:, 0] ** 2 - (big_q[:, 1:] ** 2).sum(axis=1))
    b = -big_q[:, 1:] / mass[:, None]                      # [N,3]
    gamma = big_q[:, 0] / mass
    a = 1.0 / (1.0 + gamma)
    x = sqrt_s / mass
    bq = (b[:, None, :] * q[..., 1:]).sum(axis=2)          # [N,n]
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gamma[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (
        q[..., 1:] + b[:, None, :] * q[..., 0:1] + a[:, None, None] * bq[..., None] * b[:, None, :]
    )
    return p


def _pt_eta_phi(p: np.ndarray):
    pt = np.hypot(p[..., 1], p[..., 2])
    pabs = np.sqrt(pt * pt + p[..., 3] ** 2)
    # pseudorapidity; massless partons so it equals the rapidity
    eta = 0.5 * np.log((pabs + p[..., 3]) / np.maximum(pabs - p[..., 3], 1e-300))
    phi = np.arctan2(p[..., 2], p[..., 1])
    return pt, eta, phi


def apply_cuts(finals: np.ndarray, kin: Kinematics) -> np.ndarray:
    """Boolean mask [N]: True where every final parton passes the cuts (strict)."""
    pt, eta, phi = _pt_eta_phi(finals)
    ok = np.all(pt > kin.pt_min, axis=1) & np.all(np.abs(eta) < kin.eta_max, axis=1)
    if kin.delta_r_min is not None:
        nf = finals.shape[1]
        for i in range(nf):
            for j in range(i + 1, nf):
                dphi = np.abs(phi[:, i] - phi[:, j])
                dphi = np.where(dphi > math.pi, 2.0 * math.pi - dphi, dphi)
                deta = eta[:, i] - eta[:, j]
                ok &= np.sqrt(deta * deta + dphi * dphi) > kin.delta_r_min
    return ok


def generate_events(n_events: int, n_final: int, kin: Kinematics, seed: int,
                    stream: int = 0, batch: int | None = None) -> np.ndarray:
    """Seeded events passing the cuts: float64 [n_events][2 + n_final][4].

    The generator is numpy's PCG64 seeded with (seed, stream); every event that
    fails a cut is discarded whole and replaced by a fresh draw.
    """
    rng = np.random.Generator(np.random.PCG64([seed, stream]))
    out = np.empty((n_events, 2 + n_final, 4))
    filled = 0
    batch = batch or max(1024, min(1 << 20, 4 * n_events))
    while filled < n_events:
        if kin.sqrt_s_min == kin.sqrt_s_max:
            rs = np.full(batch, kin.sqrt_s_min)
        else:
            rs = kin.sqrt_s_min + (kin.sqrt_s_max - kin.sqrt_s_min) * rng.random(batch)
        fin = rambo_massless(rng, n_final, rs)
        keep = apply_cuts(fin, kin)
        fin, rs = fin[keep], rs[keep]
        take = min(n_events - filled, fin.shape[0])
        half = 0.5 * rs[:take]
        out[filled:filled + take, 0, :] = np.stack([half, 0 * half, 0 * half, half], axis=1)
        out[filled:filled + take, 1, :] = np.stack([half, 0 * half, 0 * half, -half], axis=1)
        out[filled:filled + take, 2:, :] = fin[:take]
        filled += take
    return out


def random_helicities(n_events: int, n_ext: int, seed: int, stream: int = 0) -> np.ndarray:
    """Uniformly drawn helicity bit patterns int32 [N] (bit i set: leg i at helicity +1)."""
    rng = np.random.Generator(np.random.PCG64([seed, stream, 0x68656c]))
    return rng.integers(0, 1 << n_ext, size=n_events, dtype=np.int32)


def rambo_uniforms(n_events: int, n_final: int, kin: Kinematics, seed: int, stream: int = 0):
    """Raw inputs of one device RAMBO step: (sqrt_s float64 [N], uniforms float64 [N][n_final][4]).

    sqrt_s is uniform in [sqrt_s_min, sqrt_s_max]; the uniforms lie in (0, 1).  No cut is applied:
    an integration step gives events that fail the cuts zero weight."""
    rng = np.random.Generator(np.random.PCG64([seed, stream, 0x72616d]))
    if kin.sqrt_s_min == kin.sqrt_s_max:
        rs = np.full(n_events, float(kin.sqrt_s_min))
    else:
        rs = kin.sqrt_s_min + (kin.sqrt_s_max - kin.sqrt_s_min) * rng.random(n_events)
    u = rng.random((n_events, n_final, 4))
    u = np.where(u > 0.0, u, 0.5)          # (0, 1): log(u2 u3) stays finite
    return rs, u
