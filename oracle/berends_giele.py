"""Colour-ordered Berends-Giele recursion for pure-gluon amplitudes (oracle pin).

An independent route to the all-gluon colour-basis amplitudes: Berends and
Giele, Nucl. Phys. B306 (1988) 759, with the colour-ordered Feynman rules
for generators normalised as Tr(T^a T^b) = delta^{ab} (see e.g. L. Dixon,
TASI 1995 lectures):

  3-vertex  (i/sqrt2) [g_{nu rho}(p-q)_mu + g_{rho mu}(q-k)_nu + g_{mu nu}(k-p)_rho]
  4-vertex  (i/2) [2 g_{mu rho} g_{nu sigma} - g_{mu nu} g_{rho sigma} - g_{mu sigma} g_{nu rho}]
  propagator  -i g_{mu nu} / P^2

with all momenta flowing into the vertex and the legs in cyclic order.  The
current of a contiguous word of legs is the sum over all ways of splitting
the word into two or three contiguous sub-words.  The colour-ordered
amplitude A(w, r) closes the current of the word w of all legs but the last
(root) leg r against that leg's polarisation.

The full amplitude is M = g^{n-2} sum_w Tr(T^{w_1} ... T^{w_{n-1}} T^{r}) A(w, r),
so with t = T / sqrt2 the trace-basis amplitude of the Feynman-diagram oracle
must equal A up to one process-wide constant.
"""
from __future__ import annotations

import numpy as np

from . import lorentz as L
from .me2 import _externals, helicity_table
from .process import parse_process

_S2 = np.sqrt(2.0)


def _v3(ja, ka, jb, kb):
    kc = -(ka + kb)
    return (1j / _S2) * (jb * L.mdot(kb - kc, ja)[..., None]
                         + ja * L.mdot(kc - ka, jb)[..., None]
                         + L.mdot(ja, jb)[..., None] * (ka - kb))


def _v4(ja, jb, jc):
    return 0.5j * (2.0 * L.mdot(ja, jc)[..., None] * jb
                   - L.mdot(ja, jb)[..., None] * jc
                   - L.mdot(jb, jc)[..., None] * ja)


def bg_amplitudes(spec: str, momenta: np.ndarray, hels=None):
    """A(w, r) for every ordering w of legs 0..n-2: dict word -> [H, N]."""
    proc = parse_process(spec)
    if any(k != "g" for k in proc.kinds):
        raise ValueError("Berends-Giele pin covers pure-gluon processes")
    p = np.asarray(momenta, dtype=np.float64)
    if hels is None:
        hels = helicity_table(proc.n)
    waves, moms = _externals(proc, p, hels, None)
    cache = {}

    def current(word, prop=True):
        key = (word, prop)
        if key in cache:
            return cache[key]
        if len(word) == 1:
            res = (waves[word[0]], moms[word[0]])
        else:
            k = sum(moms[i] for i in word)
            acc = 0
            for s in range(1, len(word)):
                (ja, ka), (jb, kb) = current(word[:s]), current(word[s:])
                acc = acc + _v3(ja, ka, jb, kb)
            for s in range(1, len(word) - 1):
                for t in range(s + 1, len(word)):
                    ja, _ = current(word[:s])
                    jb, _ = current(word[s:t])
                    jc, _ = current(word[t:])
                    acc = acc + _v4(ja, jb, jc)
            if prop:
                acc = -1j * acc / L.mdot(k, k)[..., None]
            res = (acc, k)
        cache[key] = res
        return res

    import itertools
    out = {}
    legs = tuple(range(proc.n - 1))
    for w in itertools.permutations(legs):
        v, _ = current(w, prop=False)
        out[w] = L.mdot(v, waves[proc.root])
    return out


def trace_word_to_bg(word: tuple, root: int) -> tuple:
    """Rotate a cyclic trace word so that the root leg is last; drop it."""
    i = word.index(root)
    rot = word[i + 1:] + word[:i]
    return rot
