"""Colour-ordered Berends-Giele recursion: all-gluon amplitudes and one quark line (oracle pin).

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

import functools

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


def _gluon_current_fn(waves, moms):
    """Memoised colour-ordered gluon current J(word) (with its propagator) and its momentum."""
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
    return current


def bg_quark_amplitudes(spec: str, momenta: np.ndarray, hels=None):
    """Colour-ordered amplitudes of one quark line with gluons, by the Berends-Giele recursion.

    The colour factor of ordering w = (w_1 ... w_k) of the gluons is the chain
    (T^{w_1} ... T^{w_k})_{i j}, with i the colour of the row-spinor end of the line (outgoing
    quark or incoming antiquark) and j that of the column-spinor end (incoming quark or outgoing
    antiquark).  Reading the chain from the column end, the quark current that has absorbed the
    gluon word (w_s+1 ... w_k) is

        Q(w_s+1 ... w_k) = [i P/ / P^2] sum_{r} (i/sqrt2) G(w_s+1 ... w_r)/ Q(w_r+1 ... w_k)

    with Q() the external column spinor, P the momentum along the fermion arrow (column end plus
    the absorbed gluons, all momenta flowing in) and v/ = v_mu gamma^mu; the amplitude closes the
    last vertex on the row spinor without a propagator:

        A(w) = rowbar . sum_s (i/sqrt2) G(w_1 ... w_s)/ Q(w_s+1 ... w_k).

    G(u) is the colour-ordered gluon current of the trace recursion for the sub-word u read
    backwards, J(u_last ... u_first): a colour-ordered vertex lists its legs in one cyclic sense,
    which along the quark line runs against the order of the chain.

    Returns (words, dict word -> [H, N])."""
    proc = parse_process(spec)
    kinds = proc.kinds
    qi = [i for i, k in enumerate(kinds) if k == "qi"]
    qo = [i for i, k in enumerate(kinds) if k == "qo"]
    if len(qi) != 1 or len(qo) != 1:
        raise ValueError("this recursion covers processes with exactly one quark line")
    gluons = tuple(i for i, k in enumerate(kinds) if k == "g")
    p = np.asarray(momenta, dtype=np.float64)
    if hels is None:
        hels = helicity_table(proc.n)
    waves, moms = _externals(proc, p, hels, None)
    current = _gluon_current_fn(waves, moms)
    col, row = waves[qi[0]], waves[qo[0]]
    kcol = moms[qi[0]]
    vertex = lambda j, psi: (1j / _S2) * np.einsum("...ab,...b->...a", L.slash(j), psi)
    sub = lambda u: current(tuple(reversed(u)))[0]
    qcache = {}

    def quark(word):
        """Column-spinor current after absorbing the gluon word (the rightmost part of the chain)."""
        if word in qcache:
            return qcache[word]
        if not word:
            res = col
        else:
            acc = 0
            for r in range(1, len(word) + 1):
                acc = acc + vertex(sub(word[:r]), quark(word[r:]))
            q = kcol + sum(moms[i] for i in word)
            res = 1j * np.einsum("...ab,...b->...a", L.slash(q), acc) / L.mdot(q, q)[..., None]
        qcache[word] = res
        return res

    import itertools
    out = {}
    words = list(itertools.permutations(gluons))
    for w in words:
        acc = 0
        for s in range(1, len(w) + 1):
            acc = acc + vertex(sub(w[:s]), quark(w[s:]))
        out[w] = np.einsum("...a,...a->...", row, acc)
    return words, out


def trace_word_to_bg(word: tuple, root: int) -> tuple:
    """Rotate a cyclic trace word so that the root leg is last; drop it."""
    i = word.index(root)
    rot = word[i + 1:] + word[:i]
    return rot


@functools.lru_cache(maxsize=None)
def trace_colour_matrix(n: int) -> tuple:
    """Colour matrix of the single-trace basis for n gluons, averaged over two initial colours.

    Returns (words, N) with words the orderings of legs 0..n-2 (the last leg n-1 closes
    every trace) and N[w, w'] = 1/64 sum over all colours of conj(Tr(t^w t^r)) Tr(t^w' t^r),
    t = lambda/2.  The trace of n generators is built once as a tensor over its n positions;
    a relabelling of the colour indices turns the sum for (w, w') into the sum of that tensor
    against itself with the positions permuted by w^-1 w', so only (n-1)! sums are needed.
    """
    import itertools
    from .colour import _chain_tensor
    chain = _chain_tensor(n)                                  # [8]*n + [3, 3]
    tr = np.einsum("...ii->...", chain)                       # Tr(t^{b1} ... t^{bn}), [8]*n
    words = list(itertools.permutations(range(n - 1)))
    rel = {}
    for sigma in words:
        perm = list(sigma) + [n - 1]                          # trace position k holds relabelled leg perm[k]
        inv = [0] * n
        for k, leg in enumerate(perm):
            inv[leg] = k
        moved = np.transpose(tr, axes=inv)                    # moved[b] = tr[b_perm(0), ..., b_perm(n-1)]
        rel[sigma] = np.vdot(tr, moved) / 64.0
    index = {w: i for i, w in enumerate(words)}
    nmat = np.zeros((len(words), len(words)), dtype=np.complex128)
    for w in words:
        pos = {leg: k for k, leg in enumerate(w)}
        for w2 in words:
            nmat[index[w], index[w2]] = rel[tuple(pos[leg] for leg in w2)]
    return words, nmat


def bg_me2(spec: str, momenta: np.ndarray, alpha_s: float) -> np.ndarray:
    """Spin/colour averaged |M|^2 of an all-gluon process from Berends-Giele amplitudes.

    |M|^2 = 1/4 * 2^n g^(2(n-2)) * sum_h sum_{w,w'} conj(A_w) N_{w w'} A_w'
    (the full amplitude is g^(n-2) sum_w Tr(T^w T^r) A_w with T = sqrt2 t).  This route
    shares nothing with the Feynman-diagram oracle beyond the external polarisations."""
    proc = parse_process(spec)
    n = proc.n
    words, nmat = trace_colour_matrix(n)
    amps = bg_amplitudes(spec, momenta)
    a = np.stack([amps[w] for w in words], axis=-1)            # [H, N, K]
    q = np.einsum("hek,kl,hel->e", a.conj(), nmat, a).real
    g2 = 4.0 * np.pi * alpha_s
    return 0.25 * (2.0 ** n) * g2 ** (n - 2) * q
