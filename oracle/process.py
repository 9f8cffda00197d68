"""Process description and tree-diagram enumeration for the oracle.

A process string reads like "g g > g g g g", "u u~ > g g g" or "u u > u u g".
Legs are numbered 0..n-1 in the order written (initial a, b then finals).

Every external leg is typed by the kind of wavefunction it brings to the
vertex it attaches to:

* 'g'  : gluon polarisation vector;
* 'qi' : column Dirac spinor whose fermion-number arrow points into the
         diagram (incoming quark u, outgoing antiquark v);
* 'qo' : row spinor whose arrow points out of the diagram (outgoing quark u-bar,
         incoming antiquark v-bar).

Diagrams (section 2.1, eq. matrix-element; counts in Table 1) are enumerated
as trees hanging off the last leg r.  A tree for a subset S of the other legs
is either a single leg or a vertex whose children are trees over a partition
of S:

* ('ggg', A, B)          gluon from two gluon trees (unordered pair)
* ('gggg', k, A, B, C)   gluon from three gluon trees (unordered), colour
                         piece k = 0, 1, 2 of the four-gluon vertex, each
                         counted as its own diagram as the paper does
                         (section 4.2, the three colour structures)
* ('qqg_i', F, A)        'qi' spinor from a 'qi' tree F and a gluon tree A
* ('qqg_o', G, A)        'qo' spinor from a 'qo' tree G and a gluon tree A
* ('qq_g', F, G)         gluon from a 'qi' tree F and a 'qo' tree G

No sub-tree is shared between diagrams at evaluation time: each diagram is
evaluated on its own.
"""
from __future__ import annotations

import dataclasses
import functools
import itertools

FLAVOURS = ("g", "u", "u~")


@dataclasses.dataclass(frozen=True)
class OracleProcess:
    spec: str
    flavours: tuple          # per leg: 'g', 'u', 'u~'
    incoming: tuple          # per leg: True for the two initial partons
    kinds: tuple             # per leg: 'g', 'qi', 'qo'

    @property
    def n(self) -> int:
        return len(self.flavours)

    @property
    def root(self) -> int:
        return self.n - 1

    def colour_dims(self) -> tuple:
        return tuple(8 if f == "g" else 3 for f in self.flavours)

    def initial_colour_dof(self) -> int:
        """n_a n_b of eq. color-matrix: 3 per quark/antiquark, 8 per gluon."""
        return self.colour_dims()[0] * self.colour_dims()[1]


def _leg_kind(flav: str, incoming: bool) -> str:
    if flav == "g":
        return "g"
    if flav == "u":
        return "qi" if incoming else "qo"
    return "qo" if incoming else "qi"


def parse_process(spec: str) -> OracleProcess:
    lhs, rhs = spec.split(">")
    ini, fin = lhs.split(), rhs.split()
    if len(ini) != 2 or len(fin) < 2:
        raise ValueError(f"need 2 -> n>=2 partons: {spec!r}")
    flavs = tuple(ini + fin)
    for f in flavs:
        if f not in FLAVOURS:
            raise ValueError(f"unknown parton {f!r} in {spec!r}")
    inc = tuple([True, True] + [False] * len(fin))
    kinds = tuple(_leg_kind(f, i) for f, i in zip(flavs, inc))
    nqi = sum(k == "qi" for k in kinds)
    nqo = sum(k == "qo" for k in kinds)
    if nqi != nqo or nqi > 2:
        raise ValueError(f"fermion lines must close, at most two: {spec!r}")
    return OracleProcess(" ".join(ini) + " > " + " ".join(fin), flavs, inc, kinds)


def _splits2(s: frozenset):
    """Unordered partitions of s into two non-empty blocks."""
    items = sorted(s)
    first, rest = items[0], items[1:]
    for r in range(0, len(rest)):
        for comb in itertools.combinations(rest, r):
            a = frozenset((first,) + comb)
            b = s - a
            if b:
                yield a, b


def _splits2_ordered(s: frozenset):
    items = sorted(s)
    for r in range(1, len(items)):
        for comb in itertools.combinations(items, r):
            a = frozenset(comb)
            yield a, s - a


def _splits3(s: frozenset):
    """Unordered partitions of s into three non-empty blocks."""
    for a, bc in _splits2(s):
        # a holds min(s); split the remainder into two with the smaller min first
        if len(bc) < 2:
            continue
        for b, c in _splits2(bc):
            yield a, b, c


def enumerate_diagrams(proc: OracleProcess) -> list:
    """All tree diagrams, as trees over the legs other than the root leg.

    Returns a list of (tree, root_kind) where tree produces the field that
    the root leg absorbs: 'g' for a gluon root, 'qi' for a 'qo' root and
    'qo' for a 'qi' root.
    """
    kinds = proc.kinds

    @functools.lru_cache(maxsize=None)
    def trees(s: frozenset, kind: str) -> tuple:
        if len(s) == 1:
            (leg,) = tuple(s)
            return (("leg", leg),) if kinds[leg] == kind else ()
        out = []
        if kind == "g":
            for a, b in _splits2(s):
                for ta in trees(a, "g"):
                    for tb in trees(b, "g"):
                        out.append(("ggg", ta, tb))
            for a, b in _splits2_ordered(s):
                for tf in trees(a, "qi"):
                    for tg in trees(b, "qo"):
                        out.append(("qq_g", tf, tg))
            for a, b, c in _splits3(s):
                for ta in trees(a, "g"):
                    for tb in trees(b, "g"):
                        for tc in trees(c, "g"):
                            for k in range(3):
                                out.append(("gggg", k, ta, tb, tc))
        elif kind == "qi":
            for a, b in _splits2_ordered(s):
                for tf in trees(a, "qi"):
                    for ta in trees(b, "g"):
                        out.append(("qqg_i", tf, ta))
        elif kind == "qo":
            for a, b in _splits2_ordered(s):
                for tg in trees(a, "qo"):
                    for ta in trees(b, "g"):
                        out.append(("qqg_o", tg, ta))
        return tuple(out)

    root = proc.root
    need = {"g": "g", "qo": "qi", "qi": "qo"}[kinds[root]]
    rest = frozenset(range(proc.n)) - {root}
    return [(t, need) for t in trees(rest, need)]


def fermion_sign(tree, proc: OracleProcess) -> int:
    """Relative Fermi sign of a diagram from its pairing of fermion legs.

    Each fermion line runs from a 'qi' leg to a 'qo' leg.  Listing the 'qi'
    legs in increasing order, the sign is the parity of the permutation that
    sends them to their partners among the 'qo' legs in increasing order.
    """
    pairs = {}

    def walk(t):
        """Return the open fermion end ('qi' origin or 'qo' end) of the tree."""
        tag = t[0]
        if tag == "leg":
            return t[1]
        if tag == "ggg":
            walk(t[1]); walk(t[2])
            return None
        if tag == "gggg":
            walk(t[2]); walk(t[3]); walk(t[4])
            return None
        if tag in ("qqg_i", "qqg_o"):
            walk(t[2])
            return walk(t[1])
        if tag == "qq_g":
            pairs[walk(t[1])] = walk(t[2])
            return None
        raise AssertionError(tag)

    end = walk(tree)
    root = proc.root
    if proc.kinds[root] == "qo":
        pairs[end] = root
    elif proc.kinds[root] == "qi":
        pairs[root] = end
    qi = sorted(i for i, k in enumerate(proc.kinds) if k == "qi")
    qo = sorted(i for i, k in enumerate(proc.kinds) if k == "qo")
    perm = [qo.index(pairs[i]) for i in qi]
    sign = 1
    for i in range(len(perm)):
        for j in range(i + 1, len(perm)):
            if perm[i] > perm[j]:
                sign = -sign
    return sign
