"""Explicit SU(3) generators and structure constants (oracle).

t^a = lambda^a / 2 with the Gell-Mann matrices lambda^a, so that
Tr(t^a t^b) = delta^{ab}/2 and [t^a, t^b] = i f^{abc} t^c.  This is the
normalisation the paper's colour basis uses (section 2.1, eq. color-basis and
the reference given there for SU(3) conventions).
"""
from __future__ import annotations

import numpy as np

NC = 3


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, complex128 [8][3][3]."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


T = gell_mann() / 2.0


def structure_constants() -> np.ndarray:
    """f^{abc} = -2 i Tr([t^a, t^b] t^c), real float64 [8][8][8]."""
    comm = np.einsum("aij,bjk->abik", T, T) - np.einsum("bij,ajk->abik", T, T)
    f = -2j * np.einsum("abik,cki->abc", comm, T)
    assert np.max(np.abs(f.imag)) < 1e-14
    return f.real.copy()


F = structure_constants()
