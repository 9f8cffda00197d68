"""HIP source emission for one process.

Kernel shape:

* one event per lane; momenta read once per event (AoS float64 [N][n][4]);
* helicities: only configurations with leg 0 at helicity +1 are evaluated;
  the all-flipped ones give the same colour-summed |M_lambda|^2 for massless
  real kinematics, so the sum is doubled.  Quark lines have a chirality fixed
  by their end helicities; configurations breaking chirality along a line are
  structural zeros and never evaluated.  Each distinct quark-chirality pattern
  is its own straight-line block (chirality is a template constant); gluon
  helicities run in a runtime loop;
* per configuration: diagram amplitudes are emitted colour class by colour
  class; the shared currents they need are built on demand inside "groups" of
  consecutive amplitudes whose simulated register footprint stays under a
  budget.  Each group starts from opaque copies of the external momenta and
  wavefunctions, so a current shared by two groups is recomputed rather than
  held live across the whole kernel (the register file, not the arithmetic,
  is what limits these kernels);
* class sums (float64) are added into the reduced colour vector y (see
  reduce.py) held in registers, or, for large colour spaces, in LDS shared by
  the four waves of a workgroup that split the groups between them;
* the colour quadratic form y^H W y closes each configuration;
* |M|^2 = (sum over configurations) * scale, scale = 2 * 1/4 * g_s^(2(n-2)).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

from .model import Dag, Process
from .reduce import ColourSpace
from .tuned import TUNED as _TUNED_TABLE

FLOPS = {   # real floating-point operations per call, counted from the routines
    "vvv": 166, "gggg": 134, "iov": 58, "vvvx": 166, "ggggx": 134, "iovx": 58,
    "jvv": 156, "jggg": 120, "jio": 64, "fvi": 74, "fvo": 74,
    "ext": 40, "psum": 4, "inv": 8, "class_add": 4, "jamp_add": 4,
    # sum of two operands of a closing vertex (vector / spinor), plain or with a rational factor
    "sum_V": 8, "sum_W": 4, "lin_V": 16, "lin_W": 8,
}

CHUNK_FLOPS = 40000     # arithmetic per lane and configuration in one chunk function
# the same when several waves share a workgroup: finer for float32 so that eight waves balance
COOP_CHUNK_FLOPS = {"double": 40000, "float": 20000}
# ... but at most 1 / COOP_CHUNKS_PER_WAVE of a wave's share of the pattern, so that the longest-
# first assignment of chunks to waves can balance them
COOP_CHUNKS_PER_WAVE = 16
LDS_PER_CU = 160 * 1024   # bytes of LDS per compute unit (gfx950)
# resident waves per CU the workgroup shape aims for.  float32 code fits 256 registers, so two
# waves per SIMD hide each other's latency; float64 code needs more (the allocator keeps the
# excess in AGPRs instead of scratch), so one wave per SIMD with the whole register file.
TARGET_WAVES_PER_CU = {"double": 4, "float": 8}
FORCE_WAVES = 0           # if non-zero, waves per workgroup for every process and precision (for tuning)
# Each call of a chunk function saves and restores the callee-saved registers it uses (scratch
# traffic), so a wave's consecutive chunks are merged into one called function of up to this many
# chunks.  Merged functions compile more slowly; patterns with more than MERGE_MAX_PATTERN_FLOPS
# arithmetic per configuration (g g > g g g g g) keep one function per chunk so that no translation
# unit takes much longer than a quarter of an hour (merged, its float64 unit took more than 40
# minutes).
MERGE_WAVE_CHUNKS = 16
MERGE_MAX_PATTERN_FLOPS = 1_500_000
# The summed kernel runs, per pattern, one loop over the helicity configurations inside each wave's
# branch (clear the colour vector, the wave's diagram work, its colour-sum share, with the workgroup
# barriers between them), with the wave's work inlined when it is one merged function: no call per
# configuration, so no save and restore of callee-saved registers per configuration.  The loop lives
# in the kernel, not in a called function: a loop around a body of several hundred KB needs long
# branches, and in a called function those have been compiled with the return-address registers as
# their scratch pair.  Each iteration passes the lane index through an opaque copy, so the LDS
# addresses of the colour-vector rows are formed inside the loop instead of being hoisted out of it
# and spilled (measured: the float64 u u~ > 5g kernel then needs no scratch at all).  The
# sampled-helicity and test-hook kernels call the chunk functions; a tuned setting "calls" keeps one
# call per configuration in the summed kernel too.
WAVE_LOOP = True
# Diagrams of one colour class that share all operands of their closing vertex but one, and whose
# differing operands cover the same external legs (so carry the same momentum), are contracted once
# with the sum of those operands: the vertex is linear in each operand current.
MERGE_OPERANDS = True
REBALANCE_MIN = 0.02      # relative reduction of the largest wave load that a refined assignment must reach
# Column-loop unroll of the colour sum per precision (measured on u u~ > 5g: 4 for float64, 2 for mixed)
COLOUR_SUM_UNROLL = {"double": 4, "float": 2}
GROUP_BUDGET = {"double": 176, "float": 176}   # simulated live 32-bit registers per group
# How amplitudes are packed into register groups: "greedy" (whole colour classes, each group grown by
# the class that shares the most currents with it) or "classes" (first-seen class order, cut anywhere).
PLAN = "greedy"
# Per (process, precision) settings that measured faster on MI355X than the defaults above
# (gen/tuned.py, written by python -m paper_0909_5257_amd.tune): "externals": "group" rebuilds
# each external wavefunction inside every group from the LDS momenta (nothing stays live across
# groups, so a larger budget fits); the default keeps the chunk's external momenta and
# wavefunctions in registers across its groups.  "budget" replaces GROUP_BUDGET.
TUNED = dict(_TUNED_TABLE)

SIZES = {   # 32-bit registers per value
    "double": {"V": 16, "I": 8, "O": 8, "P": 8, "Q": 0, "inv": 2, "amp": 4, "pl": 8},
    "float": {"V": 8, "I": 4, "O": 4, "P": 8, "Q": 4, "inv": 1, "amp": 2, "pl": 8},
}


def _h_of_leg(proc: Process, leg: int, lam: int) -> int:
    return lam if proc.legs[leg].flavour == "u" else -lam


class Pattern:
    """One quark-chirality assignment and the gluon helicities that go with it."""

    def __init__(self, hq: dict, free_gluons: list, fixed: dict, amps: list):
        self.hq = hq
        self.free_gluons = free_gluons
        self.fixed = fixed
        self.amps = amps

    @property
    def ncfg(self):
        return 1 << len(self.free_gluons)


def _active(dag: Dag, hq: dict):
    nd = dag.nodes
    ok = {}
    for node in nd:
        if node.op == "ext":
            ok[node.id] = True
            continue
        good = all(ok[a] for a in node.args)
        if good and node.op == "jio":
            f, g = nd[node.args[0]], nd[node.args[1]]
            good = hq[f.end] == hq[g.end]
        ok[node.id] = good
    amps = []
    root = dag.proc.root
    for i, amp in enumerate(dag.amps):
        good = all(ok[a] for a in amp.args)
        if good and amp.op == "iov":
            good = hq[nd[amp.args[0]].end] == hq[root]
        elif good and amp.op == "iovx":
            good = hq[nd[amp.args[0]].end] == hq[nd[amp.args[1]].end]
        if good:
            amps.append(i)
    return amps


def patterns(dag: Dag) -> list:
    proc = dag.proc
    quarks = [l.index for l in proc.legs if l.kind != "V"]
    gluons = [l.index for l in proc.legs if l.kind == "V"]
    fixed_leg = 0   # helicity of leg 0 is fixed to +1 (flip symmetry)
    out, seen = [], set()
    for lams in itertools.product((1, -1), repeat=len(quarks)):
        lam = dict(zip(quarks, lams))
        if fixed_leg in lam and lam[fixed_leg] != 1:
            continue
        hq = {q: _h_of_leg(proc, q, lam[q]) for q in quarks}
        key = tuple(sorted(hq.items()))
        if key in seen:
            continue
        seen.add(key)
        amps = _active(dag, hq)
        if not amps:
            continue
        free = [g for g in gluons if g != fixed_leg]
        fixed = {fixed_leg: 1} if fixed_leg in gluons else {}
        out.append(Pattern(hq, free, fixed, amps))
    return out


def colour_classes(vectors: dict, amp_ids: list):
    """Group amplitudes whose accumulation vectors are proportional (first-seen order)."""
    classes, lookup = [], {}
    for i in amp_ids:
        vec = vectors[i]
        if not vec:
            continue
        k0 = min(vec)
        norm = tuple(sorted((k, v / vec[k0]) for k, v in vec.items()))
        if norm in lookup:
            ci = lookup[norm]
            classes[ci][1].append((i, vec[k0] / classes[ci][0][k0]))
        else:
            lookup[norm] = len(classes)
            classes.append((dict(vec), [(i, Fraction(1))]))
    return classes


def _lit(x) -> str:
    v = float(x)
    s = repr(v)
    if "e" not in s and "." not in s and "inf" not in s:
        s += ".0"
    return s


class _Group:
    """Straight-line code of one group of amplitudes, with register simulation."""

    def __init__(self, em, pat, prec, gid):
        self.em, self.pat, self.prec, self.gid = em, pat, prec, gid
        self.lines = []
        self.defs = {}          # value key -> (time, size)
        self.last = {}          # value key -> last use time
        self.t = 0
        self.flops = 0

    def _def(self, key, size):
        self.defs[key] = (self.t, size)
        self.last[key] = self.t
        self.t += 1

    def _use(self, key):
        self.last[key] = self.t

    def peak(self):
        ev = [0] * (self.t + 2)
        for key, (t0, size) in self.defs.items():
            t1 = self.last[key]
            if t1 > t0 and size:
                ev[t0] += size
                ev[t1] -= size
        run = peak = 0
        for x in ev:
            run += x
            peak = max(peak, run)
        return peak

    def name(self, key):
        return f"g{self.gid}_{key[0]}{'_'.join(str(x) for x in key[1:])}"

    def leg_mom(self, leg):
        """The leg's momentum: an opaque copy of the chunk's value, or read from LDS in the group."""
        key = ("pl", leg)
        if key not in self.defs:
            if self.em.group_externals[self.prec]:
                src = (f"mom4<double>{{pml[{leg}][0][lane], pml[{leg}][1][lane], pml[{leg}][2][lane], "
                       f"pml[{leg}][3][lane]}}")
            else:
                src = f"pl{leg}"
            self.lines.append(f"  const mom4<double> {self.name(key)} = fresh({src});")
            self._def(key, SIZES[self.prec]["pl"])
        self._use(key)
        return self.name(key)

    def psum(self, mask):
        key = ("P", mask)
        if key not in self.defs:
            proc = self.em.proc
            root_bit = 1 << proc.root
            if mask & root_bit and mask != root_bit:
                # a current through the root leg (closing vertex moved inwards): its momentum is minus
                # that of the complementary legs, taken that way so that every propagator invariant is
                # formed from the same legs as in a root-closed evaluation (same rounding)
                rest = ((1 << proc.n) - 1) ^ mask
                self.lines.append(f"  const mom4<double> {self.name(key)} = neg({self.psum(rest)});")
                self._def(key, SIZES[self.prec]["P"])
                self._use(key)
                return self.name(key)
            bits = [i for i in range(proc.n) if mask >> i & 1]
            if len(bits) == 1:
                i = bits[0]
                src = self.leg_mom(i)
                expr = src if proc.legs[i].eta > 0 else f"neg({src})"
            else:
                lo = 1 << bits[0]
                a, b = self.psum(lo), self.psum(mask ^ lo)
                expr = f"add({a}, {b})"
                self.flops += FLOPS["psum"]
            self.lines.append(f"  const mom4<double> {self.name(key)} = {expr};")
            self._def(key, SIZES[self.prec]["P"])
        self._use(key)
        return self.name(key)

    def qmom(self, mask):
        key = ("Q", mask)
        if key not in self.defs:
            p = self.psum(mask)
            self.lines.append(f"  const mom4<R> {self.name(key)} = to<R>({p});")
            self._def(key, SIZES[self.prec]["Q"])
        self._use(key)
        return self.name(key)

    def inv(self, mask):
        key = ("I", mask)
        if key not in self.defs:
            p = self.psum(mask)
            self.lines.append(f"  const R {self.name(key)} = inv_msq<R>({p});")
            self._def(key, SIZES[self.prec]["inv"])
            self.flops += FLOPS["inv"]
        self._use(key)
        return self.name(key)

    def node(self, i):
        key = ("c", i)
        if key in self.defs:
            self._use(key)
            return self.name(key)
        em = self.em
        nd = em.dag.nodes[i]
        h = self.pat.hq
        args = [self.node(a) for a in nd.args]
        op = nd.op
        if op == "ext" and not em.group_externals[self.prec]:
            leg = em.proc.legs[nd.leg]
            typ = "vec4<R>" if leg.kind == "V" else "wsp<R>"
            expr = f"fresh(w{leg.index})"
        elif op == "ext":
            # external wavefunction rebuilt in the group from the LDS momentum
            leg = em.proc.legs[nd.leg]
            pl = self.leg_mom(leg.index)
            if leg.kind == "V":
                typ = "vec4<R>"
                if leg.index in self.pat.fixed:
                    lam = str(self.pat.fixed[leg.index])
                else:
                    lam = f"((cfg >> {self.pat.free_gluons.index(leg.index)}) & 1 ? 1 : -1)"
                expr = em.gluon_ext(pl, lam, leg)
            elif leg.kind == "I":
                typ = "wsp<R>"
                expr = f"ixxxx0<R, {h[leg.index]}>({pl})"
            else:
                typ = "wsp<R>"
                expr = f"oxxxx0<R, {h[leg.index]}>({pl})"
            self.flops += FLOPS["ext"]
        elif op == "jvv":
            x, y = nd.args
            typ = "vec4<R>"
            expr = (f"jvvxx0<R>({args[0]}, {self.qmom(em.dag.nodes[x].mask)}, {args[1]}, "
                    f"{self.qmom(em.dag.nodes[y].mask)}, {self.inv(nd.mask)})")
        elif op == "jggg":
            typ = "vec4<R>"
            expr = f"jgggx0<R>({args[0]}, {args[1]}, {args[2]}, {self.inv(nd.mask)})"
        elif op == "jio":
            typ = "vec4<R>"
            expr = f"jioxx0<R, {h[em.dag.nodes[nd.args[0]].end]}>({args[0]}, {args[1]}, {self.inv(nd.mask)})"
        elif op == "fvi":
            typ = "wsp<R>"
            expr = f"fvixx0<R, {h[nd.end]}>({args[0]}, {args[1]}, {self.qmom(nd.mask)}, {self.inv(nd.mask)})"
        elif op == "fvo":
            typ = "wsp<R>"
            expr = f"fvoxx0<R, {h[nd.end]}>({args[0]}, {args[1]}, {self.qmom(nd.mask)}, {self.inv(nd.mask)})"
        else:
            raise AssertionError(op)
        self.flops += FLOPS.get(op, 0)
        self.lines.append(f"  const {typ} {self.name(key)} = {expr};")
        self._def(key, SIZES[self.prec][nd.kind])
        for a in nd.args:
            self._use(("c", a))
        self._use(key)
        return self.name(key)

    def class_amplitudes(self, members, acc):
        """The amplitudes (ai, fac) of one colour class, added into acc with their factors; operands
        are summed first where the emitter's merge plan says so."""
        for kind, data in self.em.merge_plan(members):
            if kind == "one":
                self.amplitude(data[0], acc, data[1])
            else:
                self.merged_amplitude(data[0], data[1], acc)

    def merged_amplitude(self, p, grp, acc):
        """One closing vertex for the diagrams grp = [(ai, fac), ...], which differ only in the
        operand at position p (same external legs): fac_0 V(..., sum_i (fac_i / fac_0) X_i, ...)."""
        em = self.em
        nd = em.dag.nodes
        a0, f0 = grp[0]
        x0 = em.dag.amps[a0].args[p]
        kind = nd[x0].kind
        typ, tag = ("vec4<R>", "V") if kind == "V" else ("wsp<R>", "W")
        cur_key, cur = ("c", x0), self.node(x0)
        for ai, f in grp[1:]:
            x = em.dag.amps[ai].args[p]
            xn = self.node(x)
            r = Fraction(f) / Fraction(f0)
            if r == 1:
                expr = f"{cur} + {xn}"
                self.flops += FLOPS["sum_" + tag]
            elif r == -1:
                expr = f"{cur} - {xn}"
                self.flops += FLOPS["sum_" + tag]
            else:
                expr = f"lin<R>({cur}, R({_lit(r)}), {xn})"
                self.flops += FLOPS["lin_" + tag]
            key = ("s", a0, ai)
            self.lines.append(f"  const {typ} {self.name(key)} = {expr};")
            self._def(key, SIZES[self.prec][kind])
            self._use(cur_key)
            self._use(("c", x))
            cur_key, cur = key, self.name(key)
        self.amplitude(a0, acc, f0, override=(p, cur, cur_key))

    def amplitude(self, ai, acc, fac, override=None):
        em = self.em
        amp = em.dag.amps[ai]
        root = em.proc.root
        nd = em.dag.nodes
        args = [override[1] if override and q == override[0] else self.node(a) for q, a in enumerate(amp.args)]
        if override:
            self._use(override[2])
        if amp.op in ("vvvx", "ggggx", "iovx"):
            self._closed_amplitude(ai, amp, args, acc, fac, override)
            return
        r = self.node(em.dag.ext[root])
        if amp.op == "vvv":
            x, y = amp.args
            expr = (f"vvvxxx<R>({args[0]}, {self.qmom(nd[x].mask)}, {args[1]}, {self.qmom(nd[y].mask)}, "
                    f"{r}, {self.qmom(1 << root)})")
        elif amp.op == "gggg":
            a, b, c = args
            order = [(a, b, c, r), (a, c, r, b), (a, r, b, c)][amp.piece]
            expr = "ggggxx<R>(" + ", ".join(order) + ")"
        else:
            expr = f"iovxx0<R, {self.pat.hq[nd[amp.args[0]].end]}>({args[0]}, {r}, {args[1]})"
        self.flops += FLOPS[amp.op] + FLOPS["class_add"]
        key = ("a", ai)
        self.lines.append(f"  const cx<R> {self.name(key)} = {expr};")
        self._def(key, SIZES[self.prec]["amp"])
        for q, a in enumerate(amp.args):
            self._use(override[2] if override and q == override[0] else ("c", a))
        self._use(("c", em.dag.ext[root]))
        self._accumulate(acc, fac, key)

    def _closed_amplitude(self, ai, amp, args, acc, fac, override=None):
        """An amplitude contracted at a vertex next to the root (Dag._reclose): every argument is an
        explicit current, the root's among them."""
        nd = self.em.dag.nodes
        if amp.op == "vvvx":
            x, y, v = amp.args
            expr = (f"vvvxxx<R>({args[0]}, {self.qmom(nd[x].mask)}, {args[1]}, {self.qmom(nd[y].mask)}, "
                    f"{args[2]}, {self.qmom(nd[v].mask)})")
        elif amp.op == "ggggx":
            expr = "ggggxx<R>(" + ", ".join(args) + ")"
        else:
            expr = f"iovxx0<R, {self.pat.hq[nd[amp.args[0]].end]}>({args[0]}, {args[1]}, {args[2]})"
        self.flops += FLOPS[amp.op] + FLOPS["class_add"]
        key = ("a", ai)
        self.lines.append(f"  const cx<R> {self.name(key)} = {expr};")
        self._def(key, SIZES[self.prec]["amp"])
        for q, a in enumerate(amp.args):
            self._use(override[2] if override and q == override[0] else ("c", a))
        self._accumulate(acc, fac, key)

    def _accumulate(self, acc, fac, key):
        an = self.name(key)
        if fac == 1:
            self.lines.append(f"  {acc}.re += double({an}.re); {acc}.im += double({an}.im);")
        elif fac == -1:
            self.lines.append(f"  {acc}.re -= double({an}.re); {acc}.im -= double({an}.im);")
        else:
            self.lines.append(f"  {acc}.re += {_lit(fac)} * double({an}.re); "
                              f"{acc}.im += {_lit(fac)} * double({an}.im);")
        self._use(key)


class Emitter:
    """Sources of one process.  With hook=True the emitter writes the test-hook kernels instead
    (me2x_*: every gluon external can be replaced by its momentum, and the reduced colour vector
    of every evaluated configuration can be written out); the hot-path kernels never carry
    that switch, so the compiler keeps folding the vanishing polarisation components."""

    def __init__(self, dag: Dag, nmat, hook: bool = False):
        self.dag = dag
        self.proc = dag.proc
        self.nmat = nmat
        self.hook = hook
        self.k = len(dag.basis)
        self.cs = ColourSpace(dag, nmat)
        self.kdim = self.cs.dim
        self.vectors = {i: self.cs.vector(a.coef) for i, a in enumerate(dag.amps)}
        self.pats = patterns(dag)
        tuned = {prec: TUNED.get((self.proc.spec, prec), {}) for prec in ("double", "float")}
        self.group_externals = {prec: tuned[prec].get("externals") == "group" for prec in tuned}
        self.budget = {prec: tuned[prec].get("budget", GROUP_BUDGET[prec]) for prec in tuned}
        self.target_waves = {prec: tuned[prec].get("waves_per_cu", TARGET_WAVES_PER_CU[prec]) for prec in tuned}
        self.kernel_loop = {prec: WAVE_LOOP and not hook and not tuned[prec].get("calls", False) for prec in tuned}
        self.nwave = {prec: self.waves_per_workgroup(prec) for prec in ("double", "float")}
        # colour-sum row blocks: the block size (a divisor of K') whose longest-first assignment to the
        # waves is best balanced (blocks of the upper triangle shrink with the row), larger on ties
        most = max(self.nwave.values())
        divs = [b for b in (8, 6, 4, 3, 2, 1) if self.kdim % b == 0]
        self.cblock = min(divs, key=lambda b: (round(self._block_owners(b, most)[1], 3), -b))
        self.flops = {"double": 0, "float": 0}
        self.algo_flops = 0
        self._merge_cache = {}
        self.stats = {}

    def merge_plan(self, members):
        """Closing vertices of one colour class's amplitudes [(ai, fac), ...]: ("merge", (p, grp))
        for diagrams grp that differ only in their operand at position p, all of one mask (so one
        momentum), contracted once with the summed operands; ("one", (ai, fac)) for the rest.
        Greedy, largest group first; deterministic."""
        key0 = tuple(members)
        if key0 in self._merge_cache:
            return self._merge_cache[key0]
        nd, amps = self.dag.nodes, self.dag.amps
        left = dict(members)
        plan = []
        while MERGE_OPERANDS and len(left) > 1:
            groups = {}
            for ai in left:
                a = amps[ai]
                for p, x in enumerate(a.args):
                    k = (a.op, a.piece, p, nd[x].mask, nd[x].kind, a.args[:p] + a.args[p + 1:])
                    groups.setdefault(k, []).append(ai)
            k, grp = max(groups.items(), key=lambda kv: (len(kv[1]), -min(kv[1])))
            if len(grp) < 2:
                break
            assert len({amps[ai].args[k[2]] for ai in grp}) == len(grp)
            plan.append(("merge", (k[2], [(ai, left[ai]) for ai in grp])))
            for ai in grp:
                del left[ai]
        plan.extend(("one", (ai, fac)) for ai, fac in left.items())
        self._merge_cache[key0] = plan
        return plan

    def _block_owners(self, bsz: int, nwave: int):
        """Longest-first assignment of the colour-sum row blocks (block j spans K' - bsz j columns of
        the upper triangle) to nwave waves: (owner of each block, max load / mean load)."""
        load, owner = [0] * nwave, []
        for j in range(self.kdim // bsz):
            wv = min(range(nwave), key=lambda v: load[v])
            owner.append(wv)
            load[wv] += self.kdim - bsz * j
        return owner, max(load) * nwave / sum(load)

    def block_table(self, prec: str) -> str:
        """__constant__ table of the row blocks each wave sums: [wave][0] = count, then the blocks."""
        nwave = self.nwave[prec]
        owner, _ = self._block_owners(self.cblock, nwave)
        rows = [[j for j, o in enumerate(owner) if o == v] for v in range(nwave)]
        width = 1 + max(len(r) for r in rows)
        name = f"CSB_{'F64' if prec == 'double' else 'F32'}"
        body = ", ".join("{" + ", ".join(str(x) for x in [len(r)] + r + [0] * (width - 1 - len(r))) + "}" for r in rows)
        return f"__constant__ int {name}[{nwave}][{width}] = {{{body}}};"

    def gluon_ext(self, pl: str, lam: str, leg) -> str:
        """Expression of one external gluon polarisation (physical momentum pl, helicity lam)."""
        out = "false" if leg.incoming else "true"
        if self.hook:
            return f"vxxxx0g<R>({pl}, {lam}, {out}, gauge == {leg.index})"
        return f"vxxxx0<R>({pl}, {lam}, {out})"

    @property
    def chunk_params(self) -> str:
        return "int cfg, int lane, int gauge" if self.hook else "int cfg, int lane"

    @property
    def chunk_args(self) -> str:
        return "cfg, lane, gauge" if self.hook else "cfg, lane"

    def slot_helicities(self) -> list:
        """Helicity bit pattern (bit i set: leg i at +1) of every evaluated configuration, in the
        order the kernels loop over them: pattern by pattern, gluon configurations in cfg order."""
        proc = self.proc
        out = []
        for pat in self.pats:
            for cfg in range(pat.ncfg):
                lam = {0: 1}
                lam.update({g: (1 if (cfg >> j) & 1 else -1) for j, g in enumerate(pat.free_gluons)})
                lam.update(pat.fixed)
                for q, hq in pat.hq.items():
                    lam[q] = hq if proc.legs[q].flavour == "u" else -hq
                out.append(sum(1 << i for i in range(proc.n) if lam[i] == 1))
        return out

    def reduction_matrix(self) -> list:
        """Exact K' x K matrix M with y = M J: the reduced colour vector the kernels accumulate,
        in terms of the colour-basis amplitudes of eq. (color-amplitude)."""
        cs = self.cs
        m = [[Fraction(0)] * self.k for _ in range(self.kdim)]
        if cs.subst is None:
            for a, p in enumerate(cs.pivots):
                m[a][p] += 1
            return m
        sel, rmat = cs.subst
        for a, s in enumerate(sel):
            m[a][cs.pivots[s]] += 1
        for b, row in rmat.items():
            for a, r in enumerate(row):
                if r != 0:
                    m[a][cs.pivots[b]] += r
        return m

    def lds_bytes(self, nwave: int) -> int:
        """Static LDS of one workgroup: momenta and colour vector of 64 events (+ partial sums)."""
        return (self.proc.n * 4 + self.kdim * 2) * 64 * 8 + (nwave * 64 * 8 if nwave > 1 else 0)

    def waves_per_workgroup(self, prec: str) -> int:
        """Fewest waves per 64-event workgroup that still put two waves on every SIMD.

        The workgroup's LDS (mostly the colour vector) limits how many workgroups share a
        compute unit; splitting each event group's diagram work over more waves raises the
        number of resident waves without raising the LDS per event."""
        if FORCE_WAVES:
            return FORCE_WAVES
        for w in (1, 2, 4, 8):
            per_cu = LDS_PER_CU // self.lds_bytes(w)
            if per_cu >= 1 and w * per_cu >= self.target_waves[prec]:
                return w
        return 8

    # ------------------------------------------------------------------ groups
    def _plan(self, pat: Pattern, prec: str):
        """Split the pattern's classes into register-bounded groups of amplitudes."""
        classes = colour_classes(self.vectors, pat.amps)
        if PLAN == "greedy":
            return classes, self._plan_greedy(pat, prec, classes)
        items = [(ci, ai, fac) for ci, (_, members) in enumerate(classes) for ai, fac in members]
        groups, cur = [], []
        budget = self.budget[prec]
        g = _Group(self, pat, prec, 0)
        for it in items:
            g.amplitude(it[1], "acc", it[2])
            if cur and g.peak() > budget:
                groups.append(cur)
                cur = [it]
                g = _Group(self, pat, prec, 0)
                g.amplitude(it[1], "acc", it[2])
            else:
                cur.append(it)
        if cur:
            groups.append(cur)
        return classes, groups

    def _plan_greedy(self, pat: Pattern, prec: str, classes) -> list:
        """Register-bounded groups of whole colour classes that share as many currents as possible.

        A group starts from the first remaining class (first-seen order) and grows by the remaining
        class whose amplitudes need the least arithmetic on top of the currents the group already
        builds (the class's closure in the DAG minus the group's), until the simulated register
        peak would exceed the budget.  Currents are recomputed only where two groups need them."""
        nd = self.dag.nodes
        root = self.dag.ext[self.proc.root]

        def cost(x):
            op = nd[x].op
            return FLOPS["ext"] if op == "ext" else FLOPS[op]
        closures = []
        for _, members in classes:
            seen, stack = set(), [root]
            for ai, _ in members:
                stack.extend(self.dag.amps[ai].args)
            while stack:
                x = stack.pop()
                if x not in seen:
                    seen.add(x)
                    stack.extend(nd[x].args)
            closures.append(seen)
        users = {}
        for ci, nodes in enumerate(closures):
            for x in nodes:
                users.setdefault(x, []).append(ci)
        full = [sum(cost(x) for x in nodes) for nodes in closures]
        remaining = set(range(len(classes)))
        budget = self.budget[prec]
        groups, pos = [], 0
        while remaining:
            while pos not in remaining:
                pos += 1
            need = {ci: full[ci] for ci in remaining}
            have, cur = set(), []
            g = _Group(self, pat, prec, 0)
            cand = pos
            while cand is not None:
                items = [(cand, ai, fac) for ai, fac in classes[cand][1]]
                g.class_amplitudes(list(classes[cand][1]), "acc")
                if cur and g.peak() > budget:
                    break
                cur.extend(items)
                remaining.discard(cand)
                del need[cand]
                for x in closures[cand] - have:
                    have.add(x)
                    c = cost(x)
                    for u in users[x]:
                        if u in need:
                            need[u] -= c
                cand = min(need, key=lambda c: (need[c], c)) if need else None
            groups.append(cur)
        return groups

    def _build(self, pat, prec, items, gid):
        g = _Group(self, pat, prec, gid)
        runs = []                       # consecutive items of one class
        for ci, ai, fac in items:
            if runs and runs[-1][0] == ci:
                runs[-1][1].append((ai, fac))
            else:
                runs.append((ci, [(ai, fac)]))
        for ci, members in runs:
            g.class_amplitudes(members, f"k{ci}")
        return g

    # ------------------------------------------------------------------ code
    def emit_pattern(self, pi: int, pat: Pattern, prec: str):
        """Chunk functions of one pattern: list of (name, source, wave, flops)."""
        proc = self.proc
        classes, groups = self._plan(pat, prec)
        last_group = {}
        for gi, items in enumerate(groups):
            for ci, _, _ in items:
                last_group[ci] = gi
        built = [self._build(pat, prec, items, gi) for gi, items in enumerate(groups)]
        # chunks: consecutive groups, cut only where no colour class is open
        nwave = self.nwave[prec]
        if nwave > 1:
            share = sum(b.flops for b in built) // (nwave * COOP_CHUNKS_PER_WAVE)
            target = max(1, min(COOP_CHUNK_FLOPS[prec], share))
        else:
            target = CHUNK_FLOPS
        chunks, cur, cur_flops = [], [], 0
        for gi, b in enumerate(built):
            cur.append(gi)
            cur_flops += b.flops
            open_cls = any(last_group[c] > gi for c, _, _ in groups[gi])
            if cur_flops >= target and not open_cls:
                chunks.append(cur)
                cur, cur_flops = [], 0
        if cur:
            chunks.append(cur)
        h = pat.hq
        prologue = []
        w = prologue.append
        if not self.group_externals[prec]:
            for leg in proc.legs:
                w(f"  const mom4<double> pl{leg.index}{{pml[{leg.index}][0][lane], pml[{leg.index}][1][lane], "
                  f"pml[{leg.index}][2][lane], pml[{leg.index}][3][lane]}};")
            for leg in proc.legs:
                if leg.kind == "V":
                    if leg.index in pat.fixed:
                        lam = str(pat.fixed[leg.index])
                    else:
                        lam = f"((cfg >> {pat.free_gluons.index(leg.index)}) & 1 ? 1 : -1)"
                    w(f"  const vec4<R> w{leg.index} = {self.gluon_ext(f'pl{leg.index}', lam, leg)};")
                elif leg.kind == "I":
                    w(f"  const wsp<R> w{leg.index} = ixxxx0<R, {h[leg.index]}>(pl{leg.index});")
                else:
                    w(f"  const wsp<R> w{leg.index} = oxxxx0<R, {h[leg.index]}>(pl{leg.index});")
        out = []
        total_flops = 0
        ext_flops = 0 if self.group_externals[prec] else FLOPS["ext"] * proc.n
        for ki, gis in enumerate(chunks):
            lines = []
            w = lines.append
            flops = 0
            for gi in gis:
                items = groups[gi]
                for ci in sorted({c for c, _, _ in items if min(g for g in range(len(groups))
                                                                 if any(x == c for x, _, _ in groups[g])) == gi}):
                    w(f"  cx<double> k{ci}{{0.0, 0.0}};")
                if self.group_externals[prec]:
                    # a group starts from LDS: no load is reused from an earlier group
                    w('  asm volatile("" ::: "memory");')
                w("  __builtin_amdgcn_sched_barrier(0);")
                lines.extend(built[gi].lines)
                flops += built[gi].flops
                for ci in sorted({c for c, _, _ in items if last_group[c] == gi}):
                    for a, sc in sorted(classes[ci][0].items()):
                        flops += FLOPS["jamp_add"]
                        if self.nwave[prec] > 1:
                            w(f"  lds_add(&yl[{a}][0][lane], {_lit(sc)} * k{ci}.re); "
                              f"lds_add(&yl[{a}][1][lane], {_lit(sc)} * k{ci}.im);")
                        else:
                            w(f"  yl[{a}][0][lane] += {_lit(sc)} * k{ci}.re; yl[{a}][1][lane] += {_lit(sc)} * k{ci}.im;")
            name = f"p{pi}_{'f64' if prec == 'double' else 'f32'}_c{ki}"
            src = (f"__device__ __noinline__ void {name}({self.chunk_params}) {{\n  using R = {prec};\n"
                   + "\n".join(prologue + lines) + "\n}\n")
            out.append([name, src, 0, flops + ext_flops, lines])
            total_flops += flops + ext_flops
        nwave = self.nwave[prec]
        if nwave > 1:
            # longest chunk first onto the least loaded wave, then moves and swaps out of the most
            # loaded wave while they lower its load (the waves meet at a barrier per configuration);
            # the refined assignment is kept only where it lowers the largest load by more than
            # REBALANCE_MIN: a different assignment is different code for the register allocator,
            # and small gains were measured to be lost to it
            load = [0] * nwave
            for c in sorted(out, key=lambda c: -c[3]):
                wv = min(range(nwave), key=lambda v: load[v])
                c[2] = wv
                load[wv] += c[3]
            lpt = [c[2] for c in out]
            lpt_max = max(load)
            for _ in range(10 * len(out)):
                top = max(range(nwave), key=lambda v: (load[v], -v))
                best, gain = None, 0
                for a in (c for c in out if c[2] == top):
                    for v in range(nwave):
                        if v == top:
                            continue
                        # move a to v, or swap it with a shorter chunk b of v
                        for b in [None] + [c for c in out if c[2] == v and c[3] < a[3]]:
                            d = a[3] - (b[3] if b else 0)
                            new_max = max(load[top] - d, load[v] + d)
                            if load[top] - new_max > gain:
                                best, gain = (a, b, v, d), load[top] - new_max
                if best is None:
                    break
                a, b, v, d = best
                a[2] = v
                if b is not None:
                    b[2] = top
                load[top] -= d
                load[v] += d
            if max(load) > (1.0 - REBALANCE_MIN) * lpt_max:
                for c, wv in zip(out, lpt):
                    c[2] = wv
        if MERGE_WAVE_CHUNKS > 1 and total_flops <= MERGE_MAX_PATTERN_FLOPS:
            # a wave's chunks in order, each in a scope of its own after one shared prologue, merged
            # into functions of up to MERGE_WAVE_CHUNKS chunks: fewer calls, fewer saves of
            # callee-saved registers, and the externals built once per call
            merged = []
            total_flops = 0
            for v in range(nwave):
                mine = [c for c in out if c[2] == v]
                for m0 in range(0, len(mine), MERGE_WAVE_CHUNKS):
                    run = mine[m0:m0 + MERGE_WAVE_CHUNKS]
                    name = f"p{pi}_{'f64' if prec == 'double' else 'f32'}_w{v}_{m0 // MERGE_WAVE_CHUNKS}"
                    body = list(prologue)
                    for c in run:
                        body.append("  {")
                        body.extend(c[4])
                        body.append("  }")
                    src = (f"__device__ __noinline__ void {name}({self.chunk_params}) {{\n  using R = {prec};\n"
                           + "\n".join(body) + "\n}\n")
                    fl = sum(c[3] - ext_flops for c in run) + ext_flops
                    merged.append([name, src, v, fl, body])
                    total_flops += fl
            out = merged
        cflops = total_flops + 2 * self.kdim * (self.kdim + 1)
        self.flops[prec] += cflops * pat.ncfg
        if prec == "double":
            self.algo_flops += self._algorithmic_flops(pat, classes) * pat.ncfg
        self.stats.setdefault(prec, []).append(
            {"pattern": pi, "amps": len(pat.amps), "groups": len(groups), "chunks": len(chunks),
             "node_evals": sum(sum(1 for k in b.defs if k[0] == "c") for b in built),
             "max_peak": max(b.peak() for b in built),
             "wave_flops": [sum(c[3] for c in out if c[2] == v) for v in range(nwave)]})
        return out

    def _algorithmic_flops(self, pat, classes) -> int:
        """Arithmetic of one configuration with every shared current built once and every closing
        vertex of the merge plan evaluated once."""
        nd = self.dag.nodes
        used, masks = set(), set()

        def visit(i):
            if i in used:
                return
            used.add(i)
            for a in nd[i].args:
                visit(a)
        for ai in pat.amps:
            for a in self.dag.amps[ai].args:
                visit(a)
        f = FLOPS["ext"] * self.proc.n
        for i in used:
            if nd[i].op != "ext":
                f += FLOPS[nd[i].op]
                masks.add(nd[i].mask)
        f += len(masks) * (FLOPS["psum"] + FLOPS["inv"])
        for _, members in classes:
            for kind, data in self.merge_plan(members):
                if kind == "one":
                    f += FLOPS[self.dag.amps[data[0]].op] + FLOPS["class_add"]
                else:
                    p, grp = data
                    a0 = self.dag.amps[grp[0][0]]
                    tag = "V" if nd[a0.args[p]].kind == "V" else "W"
                    f += FLOPS[a0.op] + FLOPS["class_add"]
                    f += sum(FLOPS[("sum_" if abs(Fraction(fac) / Fraction(grp[0][1])) == 1 else "lin_") + tag]
                             for _, fac in grp[1:])
        f += sum(len(vec) * FLOPS["jamp_add"] for vec, _ in classes)
        f += 2 * self.kdim * (self.kdim + 1)
        return f

    def colour_table(self):
        """Blocked upper-triangular W for the LDS colour sum: [K/B][K][B]."""
        k, bsz = self.kdim, self.cblock
        out = []
        for blk in range(k // bsz):
            for b in range(k):
                for a in range(bsz):
                    row = blk * bsz + a
                    if b < row:
                        v = Fraction(0)
                    elif b == row:
                        v = self.cs.w[row][b] / 2
                    else:
                        v = self.cs.w[row][b]
                    out.append(float(v))
        return out

    def helicity_map(self) -> list:
        """Per helicity bit pattern h (bit i set: leg i at +1) with leg 0 at +1: pattern << 16 | cfg, or -1.

        -1 marks a structural zero (no diagram survives the quark chiralities); patterns with
        leg 0 at -1 are looked up through their all-flipped partner, whose |M|^2 is the same."""
        proc = self.proc
        out = []
        for h in range(1 << proc.n):
            if not h & 1:
                out.append(-1)          # never read: the kernel flips such patterns first
                continue
            lam = {i: (1 if (h >> i) & 1 else -1) for i in range(proc.n)}
            code = -1
            for pi, pat in enumerate(self.pats):
                if all(_h_of_leg(proc, q, lam[q]) == hq for q, hq in pat.hq.items()):
                    cfg = sum(1 << j for j, g in enumerate(pat.free_gluons) if lam[g] == 1)
                    code = (pi << 16) | cfg
                    break
            out.append(code)
        return out

    def _kernel(self, prec: str, chunks_per_pattern, sampled: bool = False) -> list:
        """The summed kernel me2_* (every helicity configuration), with sampled=True the kernel
        me2h_* that evaluates one given helicity configuration per event, or, for a hook emitter,
        the test-hook kernel me2x_* (summed, with the gauge substitution and the colour-vector
        export)."""
        sfx = "f64" if prec == "double" else "f32"
        hel_arg = "const int* __restrict__ hel, const int* __restrict__ perm, " if sampled else ""
        args = (f"const double* __restrict__ mom, {hel_arg}int64_t nev, double* __restrict__ out, "
                "const double* __restrict__ cmat, double scale")
        if self.hook:
            args += ", int gauge, double* __restrict__ jamp"
        nwave = self.nwave[prec]
        nt = 64 * nwave
        out = []
        w = out.append
        # second bound: minimum waves per SIMD, so that the register allocator (kernel and the
        # chunk functions it calls) stays within the occupancy the LDS allows
        lds_waves_per_simd = (LDS_PER_CU // self.lds_bytes(nwave)) * nwave // 4
        min_waves = max(1, min(self.target_waves[prec] // 4, lds_waves_per_simd))
        kname = "me2x" if self.hook else ("me2h" if sampled else "me2")
        w(f"__global__ __launch_bounds__({nt}, {min_waves}) void {kname}_{sfx}({args}) {{")
        w("  const int lane = threadIdx.x & 63;")
        w("  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);")
        if sampled:
            # with perm, slot i of the launch evaluates event perm[i] (events grouped by pattern)
            w("  const int64_t slot = (int64_t)blockIdx.x * 64 + lane;")
            w("  const int64_t sc = slot < nev ? slot : nev - 1;")
            w("  const int64_t evc = perm ? (int64_t)perm[sc] : sc;")
            w("  const int64_t ev = slot < nev ? evc : nev;      // nev: no output for padding lanes")
        else:
            w("  const int64_t ev = (int64_t)blockIdx.x * 64 + lane;")
            w("  const int64_t evc = ev < nev ? ev : nev - 1;")
        w("  if (wave == 0) {")
        w("    double pm[NEXT][4];")
        w("    load_momenta<NEXT>(mom, evc, pm);")
        w("#pragma unroll")
        w("    for (int i = 0; i < NEXT; ++i)")
        w("#pragma unroll")
        w("      for (int j = 0; j < 4; ++j) pml[i][j][lane] = pm[i][j];")
        w("  }")
        if sampled:
            w("  int hcode = -2;                     // -2: helicity index out of range")
            w("  {")
            w("    int h = hel[evc];")
            w("    if (h >= 0 && h < (1 << NEXT)) {")
            w("      if (!(h & 1)) h = ~h & ((1 << NEXT) - 1);")
            w("      hcode = HMAP[h];")
            w("    }")
            w("  }")
            w("  const int my_pat = hcode >= 0 ? hcode >> 16 : -1;")
            w("  const int my_cfg = hcode >= 0 ? hcode & 0xffff : 0;")
        w("  double q = 0.0;")
        slot0 = 0
        nslots = sum(p.ncfg for p in self.pats)
        for pi, (pat, chunks) in enumerate(zip(self.pats, chunks_per_pattern)):
            if self.kernel_loop[prec] and not sampled:
                for v in range(nwave):
                    names = [c[0] for c in chunks if c[2] == v]
                    if len(names) == 1:
                        names = [names[0] + "_i"]
                    cond = ("if" if v == 0 else "} else if") + f" (wave == {v}) {{" if nwave > 1 else "{"
                    w(f"  {cond}")
                    w("#pragma unroll 1")
                    w(f"    for (int cfg = 0; cfg < {pat.ncfg}; ++cfg) {{")
                    # the lane index through an opaque copy: the LDS addresses derived from it are
                    # formed inside the loop, not hoisted out of it and kept (or spilled) for good
                    w("      const int ln = opaque_int(lane);")
                    w(f"      for (int a = threadIdx.x; a < {self.kdim * 128}; a += {nt}) (&yl[0][0][0])[a] = 0.0;")
                    w("      __syncthreads();")
                    for nm in names:
                        w(f"      {nm}(cfg, ln);")
                    w("      __syncthreads();")
                    w(f"      q += colour_sum_lds_part<{self.kdim}, {self.cblock}, {COLOUR_SUM_UNROLL[prec]}>(yl, ln, "
                      f"&CSB_{'F64' if prec == 'double' else 'F32'}[{v}][0], cmat);")
                    w("      __syncthreads();")
                    w("    }")
                w("  }")
                continue
            if sampled:
                w(f"  if (__syncthreads_or(my_pat == {pi})) {{")
                w(f"    const int cfg = my_pat == {pi} ? my_cfg : 0;")
            else:
                w("#pragma unroll 1")
                w(f"  for (int cfg = 0; cfg < {pat.ncfg}; ++cfg) {{")
            w(f"    for (int a = threadIdx.x; a < {self.kdim * 128}; a += {nt}) (&yl[0][0][0])[a] = 0.0;")
            w("    __syncthreads();")
            for v in range(nwave):
                names = [c[0] for c in chunks if c[2] == v]
                if not names:
                    continue
                if nwave > 1:
                    w(f"    if (wave == {v}) {{")
                for nm in names:
                    w(f"      {nm}({self.chunk_args});")
                if nwave > 1:
                    w("    }")
            w("    __syncthreads();")
            if self.hook:
                # reduced colour vector of this configuration: jamp[ev][slot][a][re, im]
                w("    if (jamp != nullptr && ev < nev) {")
                w(f"      double* dst = jamp + ((size_t)ev * {nslots} + {slot0} + cfg) * {2 * self.kdim};")
                w(f"      for (int a = wave; a < {self.kdim}; a += {nwave}) {{")
                w("        dst[2 * a] = yl[a][0][lane];")
                w("        dst[2 * a + 1] = yl[a][1][lane];")
                w("      }")
                w("    }")
            part = (f"colour_sum_lds_part<{self.kdim}, {self.cblock}, {COLOUR_SUM_UNROLL[prec]}>(yl, lane, "
                    f"&CSB_{'F64' if prec == 'double' else 'F32'}[wave][0], cmat)")
            if sampled:
                w(f"    const double part = {part};")
                w(f"    if (my_pat == {pi}) q += part;")
            else:
                w(f"    q += {part};")
            w("    __syncthreads();")
            w("  }")
            slot0 += pat.ncfg
        res = "(hcode == -2 ? __builtin_nan(\"\") : t * scale)" if sampled else "t * scale"
        if nwave > 1:
            w(f"  __shared__ double qsum[{nwave}][64];")
            w("  qsum[wave][lane] = q;")
            w("  __syncthreads();")
            w("  if (wave == 0) {")
            w("    double t = 0.0;")
            w(f"    for (int v = 0; v < {nwave}; ++v) t += qsum[v][lane];")
            w(f"    if (ev < nev) out[ev] = {res};")
            w("  }")
        else:
            w("  const double t = q;")
            w(f"  if (ev < nev) out[ev] = {res};")
        w("}")
        return out

    def max_launch_events(self) -> int:
        """Events one launch may cover: the grid's x dimension times the workgroup size must stay
        below 2^32 work-items, and a workgroup owns 64 events."""
        return ((1 << 32) - 1) // (64 * max(self.nwave.values())) * 64

    def _head(self) -> list:
        proc, dag = self.proc, self.dag
        head = [f"// Generated by paper_0909_5257_amd.gen for the process \"{proc.spec}\".  Do not edit.",
                f"// diagrams {len(dag.amps)}, shared currents {len(dag.nodes) - proc.n}, colour basis {self.k}, "
                f"reduced colour space {self.kdim}, helicity patterns {len(self.pats)}, "
                f"evaluated configurations {sum(p.ncfg for p in self.pats)}, waves per workgroup "
                f"{self.nwave['double']} (float64) / {self.nwave['float']} (mixed)"]
        for prec, st in self.stats.items():
            for s in st:
                head.append(f"// {prec} pattern {s['pattern']}: {s['amps']} amplitudes in {s['groups']} groups and "
                            f"{s['chunks']} chunks, {s['node_evals']} current evaluations, peak {s['max_peak']} "
                            f"registers (simulated), flops per wave {s['wave_flops']}")
        return head

    def _device_prelude(self, ns: str, with_hmap: bool) -> list:
        proc = self.proc
        lines = ['#include "heget_device.hpp"', '#include "heget_kernel_common.hpp"', "",
                 "namespace heget {", f"namespace {ns} {{", f"constexpr int NEXT = {proc.n};", "namespace {",
                 "__shared__ double pml[NEXT][4][64];        // per-event momenta of the workgroup's 64 events",
                 f"__shared__ double yl[{self.kdim}][2][64];  // reduced colour vector per event"]
        if with_hmap:
            lines.append(f"__constant__ int HMAP[{1 << proc.n}] = {{"
                         + ", ".join(str(x) for x in self.helicity_map()) + "};")
        lines.append("// colour-sum row blocks of each wave: count, then block indices")
        lines += [self.block_table("double"), self.block_table("float")]
        return lines

    def emit_hook(self) -> str:
        """The test-hook translation unit: me2x_f64 and me2x_f32 with their own chunk functions,
        and the host launcher launch_hook_<tag> (events in slices that fit one launch)."""
        assert self.hook
        proc = self.proc
        ns = f"p_{proc.tag}_hook"
        chunks = {prec: [self.emit_pattern(i, p, prec) for i, p in enumerate(self.pats)]
                  for prec in ("double", "float")}
        lines = self._head() + ["// test-hook kernels: gauge substitution and colour-vector export"]
        lines += self._device_prelude(ns, with_hmap=False)
        for prec in ("double", "float"):
            for pat_chunks in chunks[prec]:
                for c in pat_chunks:
                    lines.append(c[1])
        lines.append("}  // namespace")
        for prec in ("double", "float"):
            lines.extend(self._kernel(prec, chunks[prec]))
        lines += [f"}}  // namespace {ns}", "}  // namespace heget", ""]
        nslots = sum(p.ncfg for p in self.pats)
        per = self.max_launch_events()
        w = lines.append
        w("#if !defined(__HIP_DEVICE_COMPILE__)")
        w(f"hipError_t launch_hook_{proc.tag}(int prec, const double* mom, int64_t n, double* out, "
          "const double* cmat, double scale, int gauge, double* jamp, hipStream_t s) {")
        w(f"  for (int64_t off = 0; off < n; off += {per}LL) {{")
        w(f"    const int64_t m = n - off < {per}LL ? n - off : {per}LL;")
        w(f"    const dim3 grid((unsigned)((m + 63) / 64)), "
          f"block(prec == 0 ? {64 * self.nwave['double']} : {64 * self.nwave['float']});")
        w(f"    const double* mo = mom + off * {4 * proc.n};")
        w(f"    double* jo = jamp ? jamp + off * {nslots * 2 * self.kdim}LL : nullptr;")
        w("    if (prec == 0)")
        w(f"      hipLaunchKernelGGL(heget::{ns}::me2x_f64, grid, block, 0, s, mo, m, out + off, cmat, scale, "
          "gauge, jo);")
        w("    else")
        w(f"      hipLaunchKernelGGL(heget::{ns}::me2x_f32, grid, block, 0, s, mo, m, out + off, cmat, scale, "
          "gauge, jo);")
        w("    const hipError_t e = hipGetLastError();")
        w("    if (e != hipSuccess) return e;")
        w("  }")
        w("  return hipSuccess;")
        w("}")
        w("#endif")
        return "\n".join(lines) + "\n"

    def emit(self, with_hook: bool = False) -> dict:
        """Sources of one process: {"f64": float64 kernels + host descriptor, "f32": mixed kernels}.

        The two precisions share no device code, so they are separate translation units that
        compile in parallel; the host part launches the mixed kernels through declarations.
        with_hook: the descriptor points at launch_hook_<tag> from the separate test-hook unit."""
        assert not self.hook
        proc, dag = self.proc, self.dag
        ns = f"p_{proc.tag}"
        chunks = {prec: [self.emit_pattern(i, p, prec) for i, p in enumerate(self.pats)]
                  for prec in ("double", "float")}
        head = self._head()
        out = {}
        for prec in ("double", "float"):
            lines = list(head)
            w = lines.append
            lines += self._device_prelude(ns, with_hmap=True)
            for pat_chunks in chunks[prec]:
                for c in pat_chunks:
                    lines.append(c[1])
                    if self.kernel_loop[prec] and sum(1 for d in pat_chunks if d[2] == c[2]) == 1:
                        # the wave's only function: an inlined copy for the summed kernel's loop
                        lines.append(c[1].replace(f"__device__ __noinline__ void {c[0]}(",
                                                  f"__device__ __forceinline__ void {c[0]}_i(", 1))
            w("}  // namespace")
            lines.extend(self._kernel(prec, chunks[prec]))
            lines.extend(self._kernel(prec, chunks[prec], sampled=True))
            if prec == "double":
                args = ("const double* __restrict__ mom, int64_t nev, double* __restrict__ out, "
                        "const double* __restrict__ cmat, double scale")
                hargs = ("const double* __restrict__ mom, const int* __restrict__ hel, const int* __restrict__ perm, "
                         "int64_t nev, "
                         "double* __restrict__ out, const double* __restrict__ cmat, double scale")
                w(f"__global__ void me2_f32({args});     // in the mixed translation unit")
                w(f"__global__ void me2h_f32({hargs});")
            w("")
            w(f"}}  // namespace {ns}")
            w("}  // namespace heget")
            w("")
            if prec == "float":
                out["f32"] = "\n".join(lines) + "\n"
            else:
                out["f64"] = lines
        lines = out["f64"]
        w = lines.append
        w("#if !defined(__HIP_DEVICE_COMPILE__)")
        table = self.colour_table()
        w(f"static const double k_colour_table_{proc.tag}[] = {{" + ", ".join(_lit(x) for x in table) + "};")
        nvals = [(self.nmat[a][b].numerator, self.nmat[a][b].denominator)
                 for a in range(self.k) for b in range(self.k)]
        w(f"static const long long k_num_{proc.tag}[] = {{" + ", ".join(str(x[0]) for x in nvals) + "};")
        w(f"static const long long k_den_{proc.tag}[] = {{" + ", ".join(str(x[1]) for x in nvals) + "};")
        # exact reduction map y = M J and reduced colour matrix W (Q = y^H W y), for the test hooks
        mred = [x for row in self.reduction_matrix() for x in row]
        wred = [x for row in self.cs.w for x in row]
        for name, vals in (("red", mred), ("w", wred)):
            assert all(abs(x.numerator) < (1 << 62) and x.denominator < (1 << 62) for x in vals)
            w(f"static const long long k_{name}_num_{proc.tag}[] = {{" + ", ".join(str(x.numerator) for x in vals) + "};")
            w(f"static const long long k_{name}_den_{proc.tag}[] = {{" + ", ".join(str(x.denominator) for x in vals)
              + "};")
        slots = self.slot_helicities()
        w(f"static const int k_slot_hel_{proc.tag}[] = {{" + ", ".join(str(x) for x in slots) + "};")
        per = self.max_launch_events()
        w(f"static hipError_t launch_{proc.tag}(int prec, const double* mom, const int* hel, const int* perm, "
          f"int64_t n, double* out, const double* cmat, double scale, hipStream_t s) {{")
        w(f"  // events in slices of at most {per} (2^32 work-items per grid dimension); a permutation")
        w("  // (sampled mode, events sorted by pattern) indexes the whole batch and needs one slice")
        w(f"  if (perm != nullptr && n > {per}LL) return hipErrorInvalidValue;")
        w(f"  for (int64_t off = 0; off < n; off += {per}LL) {{")
        w(f"    const int64_t m = n - off < {per}LL ? n - off : {per}LL;")
        w(f"    const dim3 grid((unsigned)((m + 63) / 64)), "
          f"block(prec == 0 ? {64 * self.nwave['double']} : {64 * self.nwave['float']});")
        w(f"    const double* mo = mom + off * {4 * proc.n};")
        w("    if (hel == nullptr) {")
        w("      if (prec == 0)")
        w(f"        hipLaunchKernelGGL(heget::{ns}::me2_f64, grid, block, 0, s, mo, m, out + off, cmat, scale);")
        w("      else")
        w(f"        hipLaunchKernelGGL(heget::{ns}::me2_f32, grid, block, 0, s, mo, m, out + off, cmat, scale);")
        w("    } else if (perm == nullptr) {")
        w("      if (prec == 0)")
        w(f"        hipLaunchKernelGGL(heget::{ns}::me2h_f64, grid, block, 0, s, mo, hel + off, perm, m, out + off, "
          "cmat, scale);")
        w("      else")
        w(f"        hipLaunchKernelGGL(heget::{ns}::me2h_f32, grid, block, 0, s, mo, hel + off, perm, m, out + off, "
          "cmat, scale);")
        w("    } else {")
        w("      if (prec == 0)")
        w(f"        hipLaunchKernelGGL(heget::{ns}::me2h_f64, grid, block, 0, s, mom, hel, perm, n, out, cmat, scale);")
        w("      else")
        w(f"        hipLaunchKernelGGL(heget::{ns}::me2h_f32, grid, block, 0, s, mom, hel, perm, n, out, cmat, scale);")
        w("    }")
        w("    const hipError_t e = hipGetLastError();")
        w("    if (e != hipSuccess) return e;")
        w("  }")
        w("  return hipSuccess;")
        w("}")
        if with_hook:
            w(f"hipError_t launch_hook_{proc.tag}(int prec, const double* mom, int64_t n, double* out, "
              "const double* cmat, double scale, int gauge, double* jamp, hipStream_t s);")
        nhel = 2 * sum(p.ncfg for p in self.pats)
        hmap = self.helicity_map()
        pat_of = [hmap[h if h & 1 else ~h & ((1 << proc.n) - 1)] for h in range(1 << proc.n)]
        w(f"static const int k_pattern_{proc.tag}[] = {{" + ", ".join(str(c >> 16 if c >= 0 else -1) for c in pat_of)
          + "};")
        t = proc.tag
        w(f"extern const heget_proc_desc heget_desc_{t} = {{")
        w(f"  \"{proc.spec}\", {proc.n}, {len(dag.amps)}, {self.k}, {nhel}, {1 << proc.n},")
        w(f"  {len(table)}, k_colour_table_{t}, k_num_{t}, k_den_{t},")
        w(f"  {{{self.flops['double']}LL, {self.flops['float']}LL}}, {self.algo_flops}LL, launch_{t},")
        w(f"  {len(self.pats)}, k_pattern_{t},")
        w(f"  {self.kdim}, {len(slots)}, k_slot_hel_{t}, k_red_num_{t}, k_red_den_{t}, k_w_num_{t}, k_w_den_{t},")
        w(f"  {'launch_hook_' + t if with_hook else 'nullptr'}, {per}LL}};")
        w("#endif")
        out["f64"] = "\n".join(lines) + "\n"
        return out
