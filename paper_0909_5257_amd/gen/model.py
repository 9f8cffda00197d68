"""Process model and shared-current diagram DAG for the HIP generator.

A process "a b > 1 2 ... n" (section 2.1, eq. processes) is turned into

* off-shell currents, one per (subset of external legs, colour structure),
  each built once and shared by every diagram that contains it: gluon
  currents from jvvxx0 (three-gluon), the three jgggx0 pieces (four-gluon)
  and jioxx0 (quark pair); quark currents from fvixx0 / fvoxx0;
* diagram amplitudes closing the currents on a root leg with vvvxxx,
  ggggxx (three pieces) or iovxx0 (section 4, Table 4; section 2.1, eq.
  matrix-element);
* for every diagram its colour factor expanded exactly in the colour basis
  (eq. color-amplitude), from which the generator groups diagrams whose
  colour vectors are proportional ("colour classes").

Wavefunction kinds: 'V' vector (gluon), 'I' flowing-in fermion (column
spinor: incoming u, outgoing u~), 'O' flowing-out fermion (row spinor:
outgoing u, incoming u~).  Momenta of currents follow the HELAS flowing-out
convention: the slot momentum of a subset S is P_S = sum_{i in S} eta_i p_i,
eta = -1 for incoming and +1 for outgoing legs.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

from . import colour_algebra as ca

FLAVOURS = ("g", "u", "u~")
# evaluate diagrams at the vertex next to the root where that saves a current (Dag._reclose)
RECLOSE = True


@dataclasses.dataclass(frozen=True)
class Leg:
    index: int
    flavour: str
    incoming: bool

    @property
    def kind(self) -> str:
        if self.flavour == "g":
            return "V"
        if self.flavour == "u":
            return "I" if self.incoming else "O"
        return "O" if self.incoming else "I"

    @property
    def eta(self) -> int:
        return -1 if self.incoming else 1


@dataclasses.dataclass
class Process:
    spec: str
    legs: list

    @property
    def n(self):
        return len(self.legs)

    @property
    def tag(self):
        a, b = self.spec.split(">")
        conv = lambda s: "".join("ux" if f == "u~" else f for f in s.split())
        return conv(a) + "_" + conv(b)

    def kinds(self):
        return [l.kind for l in self.legs]

    @property
    def root(self) -> int:
        ks = self.kinds()
        outs = [i for i, k in enumerate(ks) if k == "O"]
        return outs[-1] if outs else self.n - 1

    @property
    def colour_dof(self):
        d = [8 if l.flavour == "g" else 3 for l in self.legs]
        return d[0] * d[1]


def parse(spec: str) -> Process:
    if ">" not in spec:
        raise ValueError("process must read like 'g g > g g g'")
    lhs, rhs = spec.split(">")
    ini, fin = lhs.split(), rhs.split()
    if len(ini) != 2 or len(fin) < 2:
        raise ValueError("need two initial and at least two final partons")
    legs = []
    for i, f in enumerate(ini + fin):
        if f not in FLAVOURS:
            raise ValueError(f"unsupported parton {f!r}")
        legs.append(Leg(i, f, i < 2))
    p = Process(" ".join(ini) + " > " + " ".join(fin), legs)
    ks = p.kinds()
    if ks.count("I") != ks.count("O") or ks.count("I") > 2:
        raise ValueError("quark lines must close (at most two)")
    return p


@dataclasses.dataclass
class Node:
    id: int
    kind: str                 # 'V', 'I', 'O'
    mask: int                 # external legs covered
    op: str                   # 'ext', 'jvv', 'jggg', 'jio', 'fvi', 'fvo'
    args: tuple               # node ids (ordered as the call takes them)
    colour: object            # colour_algebra.Poly
    end: Optional[int]        # fermion end leg (in-leg of 'I', out-leg of 'O')
    pairs: tuple              # closed fermion lines inside: ((in_leg, out_leg), ...)
    leg: Optional[int] = None


@dataclasses.dataclass
class Amp:
    op: str                   # 'vvv', 'gggg', 'iov'
    args: tuple               # node ids; the root wavefunction is implied
    colour: object
    pairs: tuple
    piece: int = 0            # for 'gggg': which of the three colour pieces
    coef: dict = None         # basis index -> integer coefficient (incl. Fermi sign)
    sign: int = 1


def _mask(s):
    m = 0
    for i in s:
        m |= 1 << i
    return m


def _splits2(items):
    first, rest = items[0], items[1:]
    for r in range(0, len(rest)):
        for comb in itertools.combinations(rest, r):
            a = (first,) + comb
            b = tuple(x for x in items if x not in a)
            if b:
                yield a, b


def _splits2_ordered(items):
    for r in range(1, len(items)):
        for comb in itertools.combinations(items, r):
            yield comb, tuple(x for x in items if x not in comb)


def _splits3(items):
    for a, bc in _splits2(items):
        if len(bc) >= 2:
            for b, c in _splits2(bc):
                yield a, b, c


class Dag:
    def __init__(self, proc: Process):
        self.proc = proc
        self.nodes: list[Node] = []
        self.by_key: dict = {}
        kinds = proc.kinds()
        root = proc.root
        self.ext = {}
        for leg in proc.legs:
            node = self._add(leg.kind, 1 << leg.index, "ext", (), self._ext_colour(leg),
                             leg.index if leg.kind != "V" else None, (), leg.index)
            self.ext[leg.index] = node.id
        rest = tuple(i for i in range(proc.n) if i != root)
        self.amps: list[Amp] = []
        self._close(rest, kinds[root])
        self._basis_and_coefficients()
        if RECLOSE:
            self._reclose()

    # ---------------------------------------------------------------- build
    def _ext_colour(self, leg):
        if leg.kind == "V":
            return ca.Poly.letter(leg.index)
        return ca.Poly.unit()

    def _add(self, kind, mask, op, args, colour, end, pairs, leg=None):
        node = Node(len(self.nodes), kind, mask, op, args, colour, end, pairs, leg)
        self.nodes.append(node)
        return node

    def currents(self, items: tuple, kind: str) -> list:
        key = (items, kind)
        if key in self.by_key:
            return self.by_key[key]
        ks = self.proc.kinds()
        out = []
        if len(items) == 1:
            if ks[items[0]] == kind:
                out = [self.ext[items[0]]]
        elif kind == "V":
            for a, b in _splits2(items):
                for x in self.currents(a, "V"):
                    for y in self.currents(b, "V"):
                        out.append(self._jvv(x, y).id)
            for a, b, c in _splits3(items):
                for x in self.currents(a, "V"):
                    for y in self.currents(b, "V"):
                        for z in self.currents(c, "V"):
                            for args in ((x, y, z), (z, x, y), (y, z, x)):
                                out.append(self._jggg(*args).id)
            for a, b in _splits2_ordered(items):
                for f in self.currents(a, "I"):
                    for g in self.currents(b, "O"):
                        out.append(self._jio(f, g).id)
        elif kind == "I":
            for a, b in _splits2_ordered(items):
                for f in self.currents(a, "I"):
                    for v in self.currents(b, "V"):
                        out.append(self._fvi(f, v).id)
        elif kind == "O":
            for a, b in _splits2_ordered(items):
                for g in self.currents(a, "O"):
                    for v in self.currents(b, "V"):
                        out.append(self._fvo(g, v).id)
        self.by_key[key] = out
        return out

    def _jvv(self, x, y):
        a, b = self.nodes[x], self.nodes[y]
        col = ca.comm(a.colour, b.colour)
        return self._add("V", a.mask | b.mask, "jvv", (x, y), col, None, a.pairs + b.pairs)

    def _jggg(self, x, y, z):
        a, b, c = self.nodes[x], self.nodes[y], self.nodes[z]
        col = -ca.comm(ca.comm(a.colour, b.colour), c.colour)
        return self._add("V", a.mask | b.mask | c.mask, "jggg", (x, y, z), col, None,
                         a.pairs + b.pairs + c.pairs)

    def _jio(self, f, g):
        a, b = self.nodes[f], self.nodes[g]
        col = ca.close_line(b.colour, a.colour, b.end, a.end)
        return self._add("V", a.mask | b.mask, "jio", (f, g), col, None,
                         a.pairs + b.pairs + ((a.end, b.end),))

    def _fvi(self, f, v):
        a, b = self.nodes[f], self.nodes[v]
        col = -(b.colour * a.colour)
        return self._add("I", a.mask | b.mask, "fvi", (f, v), col, a.end, a.pairs + b.pairs)

    def _fvo(self, g, v):
        a, b = self.nodes[g], self.nodes[v]
        col = -(a.colour * b.colour)
        return self._add("O", a.mask | b.mask, "fvo", (g, v), col, a.end, a.pairs + b.pairs)

    def _close(self, rest, root_kind):
        root = self.proc.root
        nd = self.nodes
        if root_kind == "V":
            for a, b in _splits2(rest):
                for x in self.currents(a, "V"):
                    for y in self.currents(b, "V"):
                        m = ca.comm(nd[x].colour, nd[y].colour)
                        self.amps.append(Amp("vvv", (x, y), ca.finish_trace(m, root), nd[x].pairs + nd[y].pairs))
            for a, b, c in _splits3(rest):
                for x in self.currents(a, "V"):
                    for y in self.currents(b, "V"):
                        for z in self.currents(c, "V"):
                            for piece, args in enumerate(((x, y, z), (z, x, y), (y, z, x))):
                                na, nb, nc = (nd[i] for i in args)
                                m = -ca.comm(ca.comm(na.colour, nb.colour), nc.colour)
                                self.amps.append(Amp("gggg", (x, y, z), ca.finish_trace(m, root),
                                                     na.pairs + nb.pairs + nc.pairs, piece))
            if any(k != "V" for k in self.proc.kinds()):
                raise NotImplementedError("processes with quarks close on a quark leg")
        elif root_kind == "O":
            for a, b in _splits2_ordered(rest):
                for f in self.currents(a, "I"):
                    for v in self.currents(b, "V"):
                        w = -(nd[v].colour * nd[f].colour)
                        col = ca.finish_chain(w, root, nd[f].end)
                        self.amps.append(Amp("iov", (f, v), col, nd[f].pairs + nd[v].pairs + ((nd[f].end, root),)))
        else:
            raise NotImplementedError("root leg must be a gluon or a flowing-out quark")

    # ---------------------------------------------------------------- closing vertex
    def _reclose(self):
        """Evaluate each diagram at the vertex next to the root where that saves a current.

        A diagram's amplitude is the same number whichever of its vertices the currents are
        contracted at; only the currents needed differ.  With a quark root every diagram is
        iov(F, root, J).  If F = fvi(F', G) is built for this diagram alone, the amplitude is taken
        at F's vertex instead: iovx(F', O, G) with O = fvo(root, J), the root line continued
        through J, which all diagrams with the same J share.  Otherwise, if J is built for this
        diagram alone, at J's vertex: with V = jio(F, root) (the current of the pair F, root,
        shared by all diagrams with the same F), jvv(X, Y) becomes vvvx(X, Y, V), a jggg piece
        (X, Y, Z) becomes ggggx(X, Y, Z, V) and jio(F'', O'') becomes iovx(F'', O'', V).  Colour
        factors and signs stay those of the diagram; the propagator between the two vertices
        moves from the expanded current into O or V (same invariant).  With a gluon root,
        four-gluon diagrams keep the root closure; a three-gluon diagram vvv(A, B, W) with W the
        root gluon and B (or A) built for it alone is taken at B's vertex with V = jvv(W, A) (or
        jvv(B, W)), which the cyclic, antisymmetric three-gluon vertex makes equal.  Unused
        currents are dropped and the rest renumbered."""
        nd = self.nodes
        root_ext = self.ext[self.proc.root]
        use = {}
        for node in nd:
            for a in node.args:
                use[a] = use.get(a, 0) + 1
        for amp in self.amps:
            for a in amp.args:
                use[a] = use.get(a, 0) + 1
        made = {}

        def derived(key, build):
            if key not in made:
                made[key] = build().id
            return made[key]
        expand = {"jvv": "vvvx", "jggg": "ggggx"}
        for amp in self.amps:
            if amp.op == "vvv":
                a, b = amp.args
                if nd[b].op in expand and use[b] == 1:
                    # vvv(A, B, W) = V . B with V = jvv(W, A) (cyclic three-gluon vertex)
                    v = derived(("jvv", root_ext, a), lambda: self._jvv(root_ext, a))
                    amp.op, amp.args = expand[nd[b].op], tuple(nd[b].args) + (v,)
                elif nd[a].op in expand and use[a] == 1:
                    # vvv(A, B, W) = V . A with V = jvv(B, W)
                    v = derived(("jvv", b, root_ext), lambda: self._jvv(b, root_ext))
                    amp.op, amp.args = expand[nd[a].op], tuple(nd[a].args) + (v,)
                continue
            if amp.op != "iov":
                continue
            f, j = amp.args
            if nd[f].op == "fvi" and use[f] == 1:
                fp, g = nd[f].args
                o = derived(("fvo", j), lambda: self._fvo(root_ext, j))
                amp.op, amp.args = "iovx", (fp, o, g)
            elif nd[j].op in ("jvv", "jggg", "jio") and use[j] == 1:
                v = derived(("jio", f), lambda: self._jio(f, root_ext))
                inner = nd[j].args
                amp.op = {"jvv": "vvvx", "jggg": "ggggx", "jio": "iovx"}[nd[j].op]
                amp.args = tuple(inner) + (v,)
        # keep the currents the amplitudes reach, in their order of creation
        live, stack = set(self.ext.values()), [a for amp in self.amps for a in amp.args]
        while stack:
            x = stack.pop()
            if x not in live:
                live.add(x)
                stack.extend(self.nodes[x].args)
        remap = {}
        kept = []
        for node in self.nodes:
            if node.id in live:
                remap[node.id] = len(kept)
                kept.append(node)
        for node in kept:
            node.id = remap[node.id]
            node.args = tuple(remap[a] for a in node.args)
        for amp in self.amps:
            amp.args = tuple(remap[a] for a in amp.args)
        self.ext = {leg: remap[i] for leg, i in self.ext.items()}
        self.nodes = kept
        self.by_key = {}

    # ---------------------------------------------------------------- colour
    def _basis_and_coefficients(self):
        proc = self.proc
        ks = proc.kinds()
        gluons = [i for i, k in enumerate(ks) if k == "V"]
        qi = [i for i, k in enumerate(ks) if k == "I"]
        qo = [i for i, k in enumerate(ks) if k == "O"]
        if not qi:
            self.basis = ca.basis_all_gluon(gluons)
        elif len(qi) == 1:
            self.basis = ca.basis_one_line(qo[0], qi[0], gluons)
        else:
            self.basis = ca.basis_two_lines(qi, qo, gluons)
        index = {ca.basis_key(e): i for i, e in enumerate(self.basis)}
        for amp in self.amps:
            amp.sign = _fermi_sign(amp.pairs, qi, qo)
            coef = {}
            for term, c in amp.colour.terms.items():
                k = index[ca.term_to_basis_key(term)]
                assert c[1] == 0, "colour coefficients are real with these conventions"
                coef[k] = coef.get(k, 0) + c[0] * amp.sign
            amp.coef = {k: v for k, v in coef.items() if v}

    def colour_matrix(self):
        """Exact N as a list of lists of Fractions (eq. color-matrix)."""
        k = len(self.basis)
        na = self.proc.colour_dof
        out = [[None] * k for _ in range(k)]
        for i in range(k):
            for j in range(i, k):
                v = ca.colour_matrix_element(self.basis[i], self.basis[j], 1, 1) / na
                out[i][j] = out[j][i] = v
        return out


def _fermi_sign(pairs, qi, qo):
    if len(qi) < 2:
        return 1
    partner = dict(pairs)
    perm = [qo.index(partner[i]) for i in qi]
    inv = sum(1 for i in range(len(perm)) for j in range(i + 1, len(perm)) if perm[i] > perm[j])
    return -1 if inv % 2 else 1
