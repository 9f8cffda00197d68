"""Exact SU(3) colour algebra for the process generator.

Colour factors of off-shell currents are kept as non-commutative polynomials
in the fundamental generators, with Gaussian-integer coefficients:

* a gluon current with open adjoint index e is represented by the matrix
  M = sum_e C(e) T^e, a sum of words in the external gluon letters;
* the paper's colour factors then act by plain matrix algebra, because
  i f^{abe} T^e = [T^a, T^b]:
      three-gluon current  (colour i f^{abc})      M = [M_a, M_b]
      four-gluon piece jgggx0(x, y, z)             M = -[[M_x, M_y], M_z]
      quark-gluon vertex (colour -T^a)             W -> -M_a W  or  -W M_a
  (section 4, eqs. qqg-amplitude, vvv-amplitude and the colour factors of
  the four-gluon pieces);
* a fermion line closed inside a gluon current keeps its chain with a
  bridge letter X, and the current's matrix is T^X (sum over X implied).

A term is a tuple (chains, word) where chains is a sorted tuple of closed
strands (row_leg, col_leg, word) and word is the open matrix word.

The colour matrix N_{alpha beta} = 1/(n_a n_b) sum_c T_alpha T_beta^* (eq.
color-matrix) is reduced exactly with the SU(N) Fierz identity
    sum_a (T^a)_{ij} (T^a)_{kl} = 1/2 (delta_il delta_kj - 1/N delta_ij delta_kl)
and Tr(1) = N = 3, in rational arithmetic.
"""
from __future__ import annotations

import functools
import itertools
from fractions import Fraction

NC = 3
X = "X"      # bridge letter (summed adjoint index shared by two chains)


def gi_mul(a, b):
    """Gaussian-integer product of (re, im) pairs."""
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def gi_add(a, b):
    return (a[0] + b[0], a[1] + b[1])


def gi_neg(a):
    return (-a[0], -a[1])


class Poly:
    """Sum of colour terms with Gaussian-integer coefficients."""

    __slots__ = ("terms",)

    def __init__(self, terms=None):
        self.terms = {} if terms is None else terms

    @staticmethod
    def letter(leg):
        return Poly({((), (leg,)): (1, 0)})

    @staticmethod
    def unit():
        return Poly({((), ()): (1, 0)})

    def add_term(self, key, coef):
        c = gi_add(self.terms.get(key, (0, 0)), coef)
        if c == (0, 0):
            self.terms.pop(key, None)
        else:
            self.terms[key] = c

    def scaled(self, coef):
        return Poly({k: gi_mul(v, coef) for k, v in self.terms.items()})

    def __add__(self, other):
        out = Poly(dict(self.terms))
        for k, v in other.terms.items():
            out.add_term(k, v)
        return out

    def __neg__(self):
        return self.scaled((-1, 0))

    def __sub__(self, other):
        return self + (-other)

    def __mul__(self, other):
        """Matrix product of the open words; closed chains multiply."""
        out = Poly()
        for (ca, wa), xa in self.terms.items():
            for (cb, wb), xb in other.terms.items():
                out.add_term((tuple(sorted(ca + cb)), wa + wb), gi_mul(xa, xb))
        return out


def comm(a: Poly, b: Poly) -> Poly:
    return a * b - b * a


def close_line(w_out: Poly, w_in: Poly, out_leg: int, in_leg: int) -> Poly:
    """Gluon current from a fermion pair: chain -(W_out T^X W_in) and matrix T^X."""
    out = Poly()
    for (ca, wa), xa in w_out.terms.items():
        for (cb, wb), xb in w_in.terms.items():
            assert X not in wa + wb, "at most one closed fermion line per current"
            chain = (out_leg, in_leg, wa + (X,) + wb)
            out.add_term((tuple(sorted(ca + cb + (chain,))), (X,)), gi_neg(gi_mul(xa, xb)))
    return out


def finish_chain(w: Poly, out_leg: int, in_leg: int) -> Poly:
    """Amplitude colour of an open line closed at the root: the chain itself."""
    out = Poly()
    for (ca, wa), xa in w.terms.items():
        out.add_term((tuple(sorted(ca + ((out_leg, in_leg, wa),))), ()), xa)
    return out


def finish_trace(m: Poly, root_leg: int) -> Poly:
    """Amplitude colour 2 Tr(M T^r) of a gluon current closed on the root gluon."""
    out = Poly()
    for (ca, wa), xa in m.terms.items():
        assert not ca
        out.add_term(((), wa + (root_leg,)), gi_mul(xa, (2, 0)))
    return out


# ------------------------------------------------------------------ basis

def basis_all_gluon(gluons):
    first, rest = gluons[0], gluons[1:]
    return [(("T", (first,) + perm),) for perm in itertools.permutations(rest)]


def basis_one_line(out_leg, in_leg, gluons):
    return [((out_leg, in_leg, perm),) for perm in itertools.permutations(gluons)]


def basis_two_lines(qi, qo, gluons):
    out = []
    for pairing in (dict(zip(qi, qo)), dict(zip(qi, qo[::-1]))):
        for r in range(len(gluons) + 1):
            for g1 in itertools.combinations(gluons, r):
                g2 = [g for g in gluons if g not in g1]
                for w1 in itertools.permutations(list(g1) + [X]):
                    for w2 in itertools.permutations(g2 + [X]):
                        out.append(((pairing[qi[0]], qi[0], tuple(w1)), (pairing[qi[1]], qi[1], tuple(w2))))
    return out


def canonical_trace(word):
    """Rotate a trace word so that its smallest letter comes first."""
    i = word.index(min(word))
    return word[i:] + word[:i]


def term_to_basis_key(term):
    """Map an amplitude colour term to the key used for basis lookup."""
    chains, word = term
    if word:                                  # all-gluon trace
        assert not chains
        return (("T", canonical_trace(word)),)
    return tuple(sorted(chains, key=lambda c: c[1]))


def basis_key(elem):
    if elem[0][0] == "T":
        return (("T", canonical_trace(elem[0][1])),)
    return tuple(sorted(elem, key=lambda c: c[1]))


# ------------------------------------------------------------------ Fierz

def _canon(traces):
    """Canonical form of a product of traces: relabel letters, rotate, sort."""
    traces = [t for t in traces]
    # relabel letters in order of first appearance after a provisional sort
    best = None
    for _ in range(2):
        order = {}
        for t in sorted(traces, key=lambda t: (len(t), t)):
            for l in t:
                if l not in order:
                    order[l] = len(order)
        rel = [tuple(order[l] for l in t) for t in traces]
        rel = [min(t[i:] + t[:i] for i in range(len(t))) if t else () for t in rel]
        cand = tuple(sorted(rel, key=lambda t: (len(t), t)))
        if best is None or cand < best:
            best = cand
        traces = list(cand)
    return best


@functools.lru_cache(maxsize=None)
def _reduce(traces) -> Fraction:
    """Value of a product of traces in which every letter appears exactly twice."""
    traces = list(traces)
    for ti, t in enumerate(traces):
        if t:
            break
    else:
        return Fraction(NC) ** len(traces)
    letter = traces[ti][0]
    # locate its second occurrence
    pos = [(i, j) for i, t in enumerate(traces) for j, l in enumerate(t) if l == letter]
    assert len(pos) == 2, traces
    (i1, j1), (i2, j2) = pos
    half = Fraction(1, 2)
    inv = Fraction(1, 2 * NC)
    rest = [t for k, t in enumerate(traces) if k not in (i1, i2)]
    if i1 == i2:
        t = traces[i1]
        a, b, c = t[:j1], t[j1 + 1:j2], t[j2 + 1:]
        xw, yw = c + a, b                         # Tr(X T Y T)
        v1 = _reduce(_canon(rest + [xw, yw]))
        v2 = _reduce(_canon(rest + [xw + yw]))
        return half * v1 - inv * v2
    t1, t2 = traces[i1], traces[i2]
    xw = t1[j1 + 1:] + t1[:j1]                    # Tr(X T)
    yw = t2[j2 + 1:] + t2[:j2]                    # Tr(Y T)
    v1 = _reduce(_canon(rest + [xw + yw]))
    v2 = _reduce(_canon(rest + [xw, yw]))
    return half * v1 - inv * v2


def _strands_to_traces(strands):
    """Join (row, col, word) strands into closed traces by matching indices."""
    pending = list(strands)
    traces = []
    while pending:
        row, col, word = pending.pop(0)
        if row is None:
            traces.append(tuple(word))
            continue
        start, cur, acc = row, col, list(word)
        while cur != start:
            k = next(k for k, s in enumerate(pending) if s[0] == cur)
            r, c, w = pending.pop(k)
            acc += list(w)
            cur = c
        traces.append(tuple(acc))
    return traces


def colour_matrix_element(ea, eb, n_a, n_b) -> Fraction:
    """N_{alpha beta} = 1/(n_a n_b) sum_c T_alpha T_beta^* for two basis elements."""
    strands = []
    for s in ea:
        if s[0] == "T":
            strands.append((None, None, tuple(("a", l) for l in s[1])))
        else:
            strands.append((("o", s[0]), ("i", s[1]), tuple(("a", l) for l in s[2])))
    for s in eb:
        # complex conjugate: transpose and reverse the word; rename the bridge
        if s[0] == "T":
            strands.append((None, None, tuple(("b" if l == X else "a", l) for l in reversed(s[1]))))
        else:
            strands.append((("i", s[1]), ("o", s[0]),
                            tuple(("b" if l == X else "a", l) for l in reversed(s[2]))))
    traces = _strands_to_traces(strands)
    ids = {}
    traces = [tuple(ids.setdefault(l, len(ids)) for l in t) for t in traces]
    return _reduce(_canon(traces)) / (n_a * n_b)
