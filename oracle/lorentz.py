"""External wavefunctions and Feynman-rule vertices with explicit Dirac matrices (oracle).

Conventions (textbook QCD, covariant derivative D = d - i g A^a t^a,
Feynman gauge, metric (+,-,-,-), chiral representation of the gamma matrices):

* quark-gluon vertex            i g gamma^mu t^a_{ij}
* three-gluon vertex            g f^{abc} [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu
                                           + g^{rho mu}(q-k)^nu], momenta incoming
* four-gluon vertex             -i g^2 [f^{abe}f^{cde}(g^{mu rho}g^{nu sigma} - g^{mu sigma}g^{nu rho})
                                        + f^{ace}f^{bde}(g^{mu nu}g^{rho sigma} - g^{mu sigma}g^{nu rho})
                                        + f^{ade}f^{bce}(g^{mu nu}g^{rho sigma} - g^{mu rho}g^{nu sigma})]
* gluon propagator              -i g^{mu nu} / q^2
* quark propagator              i qslash / q^2  (q along the fermion arrow)

The colour factors are applied separately (colour module); here only the
Lorentz and Dirac parts appear.  The paper states its own HELAS conventions for
the gluon self-couplings in section 4 (eqs. vvv-lagrangian and following);
they differ from these by one overall phase per diagram class that cancels
in |M|^2.

Massless external states of momentum p, with polar angle theta and azimuth
phi of the three-momentum:

* helicity spinors  xi_+ = (cos(theta/2), e^{i phi} sin(theta/2)),
                    xi_- = (-e^{-i phi} sin(theta/2), cos(theta/2)),
  u(p,+) = sqrt(2E) (0, xi_+),  u(p,-) = sqrt(2E) (xi_-, 0)  (chiral basis);
* antiquark spinor v(p, lambda) = u(p, -lambda): physical helicity lambda of
  the antiparticle, opposite chirality;
* polarisation eps(k, lambda) = (0, (-lambda theta_hat - i phi_hat)/sqrt(2)).
"""
from __future__ import annotations

import numpy as np

SIGMA = np.array([
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=np.complex128)

GAMMA = np.zeros((4, 4, 4), dtype=np.complex128)
GAMMA[0][:2, 2:] = np.eye(2)
GAMMA[0][2:, :2] = np.eye(2)
for _k in range(3):
    GAMMA[_k + 1][:2, 2:] = SIGMA[_k]
    GAMMA[_k + 1][2:, :2] = -SIGMA[_k]

METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


def mdot(a, b):
    """Minkowski product of contravariant 4-vectors (no complex conjugation)."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def slash(v):
    """v_mu gamma^mu as a [..., 4, 4] matrix."""
    low = v * np.array([1.0, -1.0, -1.0, -1.0])
    return np.einsum("...m,mij->...ij", low, GAMMA)


def angles(p):
    pt = np.hypot(p[..., 1], p[..., 2])
    theta = np.arctan2(pt, p[..., 3])
    phi = np.where(pt > 0, np.arctan2(p[..., 2], p[..., 1]), 0.0)
    return theta, phi


def polarisation(p, lam):
    """eps^mu(p, lambda) for lambda = +1 / -1: complex [..., 4]."""
    theta, phi = angles(p)
    th_hat = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], axis=-1)
    ph_hat = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=-1)
    eps = np.zeros(p.shape[:-1] + (4,), dtype=np.complex128)
    eps[..., 1:] = (-lam * th_hat - 1j * ph_hat) / np.sqrt(2.0)
    return eps


def spinor_u(p, lam):
    """Massless Dirac spinor u(p, lambda) (column), complex [..., 4]."""
    theta, phi = angles(p)
    norm = np.sqrt(2.0 * p[..., 0])
    out = np.zeros(p.shape[:-1] + (4,), dtype=np.complex128)
    if lam > 0:
        out[..., 2] = norm * np.cos(theta / 2)
        out[..., 3] = norm * np.exp(1j * phi) * np.sin(theta / 2)
    else:
        out[..., 0] = -norm * np.exp(-1j * phi) * np.sin(theta / 2)
        out[..., 1] = norm * np.cos(theta / 2)
    return out


def spinor_v(p, lam):
    return spinor_u(p, -lam)


def dirac_bar(psi):
    """psi^dagger gamma^0 as a row spinor."""
    return np.einsum("...i,ij->...j", psi.conj(), GAMMA[0])


# ---------------------------------------------------------------- vertices

def v_ggg(ja, ka, jb, kb, g):
    """Three-gluon vertex contracted with legs a, b: upper-index vector on the third leg.

    ka, kb: momenta flowing into the vertex along legs a and b.
    """
    kc = -(ka + kb)
    return g * (mdot(ja, jb)[..., None] * (ka - kb)
                + jb * mdot(kb - kc, ja)[..., None]
                + ja * mdot(kc - ka, jb)[..., None])


def v_gggg(piece, ja, jb, jc, g):
    """One colour piece of the four-gluon vertex contracted with legs a, b, c."""
    if piece == 0:
        val = mdot(ja, jc)[..., None] * jb - mdot(jb, jc)[..., None] * ja
    elif piece == 1:
        val = mdot(ja, jb)[..., None] * jc - mdot(jb, jc)[..., None] * ja
    else:
        val = mdot(ja, jb)[..., None] * jc - mdot(ja, jc)[..., None] * jb
    return -1j * g * g * val


def v_qqg_col(psi, j, g):
    """i g jslash psi (column spinor out)."""
    return 1j * g * np.einsum("...ij,...j->...i", slash(j), psi)


def v_qqg_row(psibar, j, g):
    """i g psibar jslash (row spinor out)."""
    return 1j * g * np.einsum("...i,...ij->...j", psibar, slash(j))


def v_qq_g(psi, psibar, g):
    """i g psibar gamma^mu psi (upper index mu)."""
    return 1j * g * np.einsum("...i,mij,...j->...m", psibar, GAMMA, psi)


def prop_gluon(v, q):
    return -1j * v / mdot(q, q)[..., None]


def prop_quark_col(v, q):
    """i qslash v / q^2, q along the fermion arrow."""
    return 1j * np.einsum("...ij,...j->...i", slash(q), v) / mdot(q, q)[..., None]


def prop_quark_row(v, q):
    """i v qslash / q^2, q along the fermion arrow."""
    return 1j * np.einsum("...i,...ij->...j", v, slash(q)) / mdot(q, q)[..., None]
