"""HIP source emission for one process.

Kernel shape (one event per lane, one wavefront per workgroup):

* momenta are read once per event (AoS float64 [N][n][4]);
* helicities: only configurations with leg 0 at helicity +1 are evaluated,
  the all-flipped ones give the same colour-summed |M_lambda|^2 for massless
  real kinematics, so the sum is doubled.  Quark lines have a chirality fixed
  by their end helicities; configurations that break chirality along a line
  are structural zeros and never evaluated.  Each distinct quark-chirality
  pattern is its own straight-line block (chirality is a template constant);
  gluon helicities run in a runtime loop;
* per configuration: external wavefunctions, shared currents (each once),
  diagram amplitudes summed per colour class, JAMP accumulation in float64
  (registers for small colour bases, LDS for large ones), and the colour
  quadratic form sum_{ab} J_a N_ab J_b^* with N read from a device table;
* |M|^2 = (sum over configurations) * scale with scale = 2 * 1/4 * g_s^(2(n-2)).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

from .model import Dag, Process

FLOPS = {   # real floating-point operations per call, counted from the routines
    "vvv": 166, "gggg": 134, "iov": 58,
    "jvv": 156, "jggg": 120, "jio": 64, "fvi": 74, "fvo": 74,
    "ext": 40, "subset": 12, "class_add": 4, "jamp_add": 4,
}

REG_JAMP_MAX = 24     # colour bases up to this size keep J in registers
COLOUR_BLOCK = 8      # rows of the colour quadratic form handled per pass


def _h_of_leg(proc: Process, leg: int, lam: int) -> int:
    return lam if proc.legs[leg].flavour == "u" else -lam


class Pattern:
    """One quark-chirality assignment and the gluon helicities that go with it."""

    def __init__(self, hq: dict, free_gluons: list, fixed: dict, nodes: list, amps: list):
        self.hq = hq                      # quark leg -> chirality
        self.free_gluons = free_gluons    # gluon legs whose helicity the cfg bits set
        self.fixed = fixed                # gluon leg -> fixed helicity
        self.nodes = nodes                # active node ids
        self.amps = amps                  # active amp indices

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
        if good:
            amps.append(i)
    return ok, amps


def patterns(dag: Dag) -> list:
    proc = dag.proc
    quarks = [l.index for l in proc.legs if l.kind != "V"]
    gluons = [l.index for l in proc.legs if l.kind == "V"]
    fixed_leg = 0   # helicity of leg 0 is fixed to +1 (flip symmetry)
    out = []
    seen = set()
    for lams in itertools.product((1, -1), repeat=len(quarks)):
        lam = dict(zip(quarks, lams))
        if fixed_leg in lam and lam[fixed_leg] != 1:
            continue
        hq = {q: _h_of_leg(proc, q, lam[q]) for q in quarks}
        key = tuple(sorted(hq.items()))
        if key in seen:
            continue
        seen.add(key)
        ok, amps = _active(dag, hq)
        if not amps:
            continue
        free = [g for g in gluons if g != fixed_leg]
        fixed = {fixed_leg: 1} if fixed_leg in gluons else {}
        out.append(Pattern(hq, free, fixed, [i for i, v in ok.items() if v], amps))
    return out


def colour_classes(dag: Dag, amp_ids: list):
    """Group amplitudes whose colour vectors are proportional; keep first-seen order."""
    classes = []          # list of (vector dict, [(amp id, factor Fraction)])
    lookup = {}
    for i in amp_ids:
        coef = dag.amps[i].coef
        if not coef:
            continue
        k0 = min(coef)
        norm = tuple(sorted((k, Fraction(v, coef[k0])) for k, v in coef.items()))
        if norm in lookup:
            ci = lookup[norm]
            base = classes[ci][0]
            classes[ci][1].append((i, Fraction(coef[k0], base[k0])))
        else:
            lookup[norm] = len(classes)
            classes.append((dict(coef), [(i, Fraction(1))]))
    return classes


def _lit(x) -> str:
    v = float(x)
    s = repr(v)
    if "e" not in s and "." not in s and "inf" not in s:
        s += ".0"
    return s


class Emitter:
    def __init__(self, dag: Dag, nmat):
        self.dag = dag
        self.proc = dag.proc
        self.nmat = nmat
        self.k = len(dag.basis)
        self.pats = patterns(dag)
        self.reg_jamp = self.k <= REG_JAMP_MAX
        self.flops_per_event = 0

    # ------------------------------------------------------------ helpers
    def _mask_name(self, m):
        return f"{m:x}"

    def emit_pattern(self, pi: int, pat: Pattern) -> str:
        dag, proc = self.dag, self.proc
        nd = dag.nodes
        out = []
        w = out.append
        done_p, done_q, done_i = set(), set(), set()
        flops = 0

        def need_p(m):
            nonlocal flops
            if m in done_p:
                return f"P{self._mask_name(m)}"
            bits = [i for i in range(proc.n) if m >> i & 1]
            if len(bits) == 1:
                i = bits[0]
                eta = proc.legs[i].eta
                sgn = "" if eta > 0 else "-"
                w(f"  const mom4<double> P{self._mask_name(m)}{{{sgn}pm[{i}][0], {sgn}pm[{i}][1], "
                  f"{sgn}pm[{i}][2], {sgn}pm[{i}][3]}};")
            else:
                lo = 1 << bits[0]
                a, b = need_p(lo), need_p(m ^ lo)
                w(f"  const mom4<double> P{self._mask_name(m)} = add({a}, {b});")
                flops += 4
            done_p.add(m)
            return f"P{self._mask_name(m)}"

        def need_q(m):
            name = f"Q{self._mask_name(m)}"
            if m not in done_q:
                p = need_p(m)
                w(f"  const mom4<R> {name} = to<R>({p});")
                done_q.add(m)
            return name

        def need_is(m):
            nonlocal flops
            name = f"I{self._mask_name(m)}"
            if m not in done_i:
                p = need_p(m)
                w(f"  const R {name} = R(1.0 / msq({p}));")
                done_i.add(m)
                flops += 8
            return name

        emitted = set()
        h = pat.hq

        def var(i):
            return f"c{i}"

        def emit_node(i):
            nonlocal flops
            if i in emitted:
                return
            node = nd[i]
            for a in node.args:
                emit_node(a)
            op = node.op
            if op == "ext":
                leg = proc.legs[node.leg]
                pl = f"pl{leg.index}"
                if leg.kind == "V":
                    if leg.index in pat.fixed:
                        lam = str(pat.fixed[leg.index])
                    else:
                        bit = pat.free_gluons.index(leg.index)
                        lam = f"((cfg >> {bit}) & 1 ? 1 : -1)"
                    w(f"  const vec4<R> {var(i)} = vxxxx0<R>({pl}, {lam}, {'false' if leg.incoming else 'true'});")
                elif leg.kind == "I":
                    w(f"  const wsp<R> {var(i)} = ixxxx0<R, {h[leg.index]}>({pl});")
                else:
                    w(f"  const wsp<R> {var(i)} = oxxxx0<R, {h[leg.index]}>({pl});")
                flops += FLOPS["ext"]
            elif op == "jvv":
                x, y = node.args
                w(f"  const vec4<R> {var(i)} = jvvxx0<R>({var(x)}, {need_q(nd[x].mask)}, {var(y)}, "
                  f"{need_q(nd[y].mask)}, {need_is(node.mask)});")
                flops += FLOPS["jvv"]
            elif op == "jggg":
                x, y, z = node.args
                w(f"  const vec4<R> {var(i)} = jgggx0<R>({var(x)}, {var(y)}, {var(z)}, {need_is(node.mask)});")
                flops += FLOPS["jggg"]
            elif op == "jio":
                f, g = node.args
                w(f"  const vec4<R> {var(i)} = jioxx0<R, {h[nd[f].end]}>({var(f)}, {var(g)}, {need_is(node.mask)});")
                flops += FLOPS["jio"]
            elif op == "fvi":
                f, v = node.args
                w(f"  const wsp<R> {var(i)} = fvixx0<R, {h[node.end]}>({var(f)}, {var(v)}, "
                  f"{need_q(node.mask)}, {need_is(node.mask)});")
                flops += FLOPS["fvi"]
            elif op == "fvo":
                g, v = node.args
                w(f"  const wsp<R> {var(i)} = fvoxx0<R, {h[node.end]}>({var(g)}, {var(v)}, "
                  f"{need_q(node.mask)}, {need_is(node.mask)});")
                flops += FLOPS["fvo"]
            else:
                raise AssertionError(op)
            emitted.add(i)

        root = proc.root
        w(f"  // quark chiralities: {', '.join(f'leg {q}: {v:+d}' for q, v in sorted(h.items())) or 'none'}")
        for leg in proc.legs:
            w(f"  const mom4<double> pl{leg.index}{{pm[{leg.index}][0], pm[{leg.index}][1], "
              f"pm[{leg.index}][2], pm[{leg.index}][3]}};")
        if self.reg_jamp:
            w(f"  double jr[{self.k}], ji[{self.k}];")
            w(f"#pragma unroll")
            w(f"  for (int a = 0; a < {self.k}; ++a) {{ jr[a] = 0.0; ji[a] = 0.0; }}")
        else:
            w(f"#pragma unroll 8")
            w(f"  for (int a = 0; a < {self.k}; ++a) jl[a][lane] = make_double2(0.0, 0.0);")

        emit_node(dag.ext[root])
        for cls_i, (vec, members) in enumerate(colour_classes(dag, pat.amps)):
            kk = f"k{cls_i}"
            w(f"  // colour class {cls_i}")
            w(f"  cx<double> {kk}{{0.0, 0.0}};")
            for ai, fac in members:
                amp = dag.amps[ai]
                for a in amp.args:
                    emit_node(a)
                if amp.op == "vvv":
                    x, y = amp.args
                    expr = (f"vvvxxx<R>({var(x)}, {need_q(nd[x].mask)}, {var(y)}, {need_q(nd[y].mask)}, "
                            f"{var(dag.ext[root])}, {need_q(1 << root)})")
                elif amp.op == "gggg":
                    x, y, z = amp.args
                    r = var(dag.ext[root])
                    order = [(x, y, z, r), (x, z, r, y), (x, r, y, z)][amp.piece]
                    expr = "ggggxx<R>(" + ", ".join(o if isinstance(o, str) else var(o) for o in order) + ")"
                else:
                    f, v = amp.args
                    expr = f"iovxx0<R, {h[nd[f].end]}>({var(f)}, {var(dag.ext[root])}, {var(v)})"
                flops += FLOPS[amp.op] + FLOPS["class_add"]
                w(f"  const cx<R> a{ai} = {expr};")
                if fac == 1:
                    w(f"  {kk}.re += double(a{ai}.re); {kk}.im += double(a{ai}.im);")
                elif fac == -1:
                    w(f"  {kk}.re -= double(a{ai}.re); {kk}.im -= double(a{ai}.im);")
                else:
                    w(f"  {kk}.re += {_lit(fac)} * double(a{ai}.re); {kk}.im += {_lit(fac)} * double(a{ai}.im);")
            for a, s in sorted(vec.items()):
                flops += FLOPS["jamp_add"]
                if self.reg_jamp:
                    w(f"  jr[{a}] += {_lit(s)} * {kk}.re; ji[{a}] += {_lit(s)} * {kk}.im;")
                else:
                    w(f"  {{ double2 t = jl[{a}][lane]; t.x += {_lit(s)} * {kk}.re; t.y += {_lit(s)} * {kk}.im; "
                      f"jl[{a}][lane] = t; }}")
        # colour sum
        if self.reg_jamp:
            w("  double q = 0.0;")
            for a in range(self.k):
                terms_r, terms_i = [], []
                for b in range(a, self.k):
                    v = self.nmat[a][b] * (Fraction(1, 2) if a == b else 1)
                    if v == 0:
                        continue
                    terms_r.append(f"{_lit(v)} * jr[{b}]")
                    terms_i.append(f"{_lit(v)} * ji[{b}]")
                if terms_r:
                    w(f"  q += jr[{a}] * ({' + '.join(terms_r)}) + ji[{a}] * ({' + '.join(terms_i)});")
            w("  return 2.0 * q;")
        else:
            w(f"  return colour_sum_lds<{self.k}, {COLOUR_BLOCK}>(jl, lane, cmat);")
        flops += 2 * self.k * (self.k + 1)
        self.flops_per_event += flops * pat.ncfg
        body = "\n".join(out)
        jarg = "" if self.reg_jamp else ", double2 (*jl)[64], int lane, const double* __restrict__ cmat"
        return (f"template <class R>\n__device__ __forceinline__ double pattern{pi}("
                f"const double (&pm)[NEXT][4], int cfg{jarg}) {{\n{body}\n}}\n")

    def colour_table(self):
        """Blocked upper-triangular colour matrix for colour_sum_lds: [K/B][K][B]."""
        k, bsz = self.k, COLOUR_BLOCK
        out = []
        for blk in range(k // bsz):
            for b in range(k):
                for a in range(bsz):
                    row = blk * bsz + a
                    if b < row:
                        v = Fraction(0)
                    elif b == row:
                        v = self.nmat[row][b] / 2
                    else:
                        v = self.nmat[row][b]
                    out.append(float(v))
        return out

    def emit(self) -> str:
        proc, dag = self.proc, self.dag
        ns = f"p_{proc.tag}"
        pats = [self.emit_pattern(i, p) for i, p in enumerate(self.pats)]
        kern_args = "const double* __restrict__ mom, int64_t nev, double* __restrict__ out, " \
                    "const double* __restrict__ cmat, double scale"
        lines = []
        w = lines.append
        w(f"// Generated by paper_0909_5257_amd.gen for the process \"{proc.spec}\".  Do not edit.")
        w(f"// diagrams {len(dag.amps)}, shared currents {len(dag.nodes) - proc.n}, colour basis {self.k}, "
          f"helicity patterns {len(self.pats)}, evaluated configurations {sum(p.ncfg for p in self.pats)}")
        w('#include "heget_device.hpp"')
        w('#include "heget_kernel_common.hpp"')
        w("")
        w("namespace heget {")
        w(f"namespace {ns} {{")
        w(f"constexpr int NEXT = {proc.n};")
        w(f"constexpr int NCOL = {self.k};")
        w("")
        for p in pats:
            w(p)
        w("template <class R>")
        w(f"__global__ __launch_bounds__(64) void me2_kernel({kern_args}) {{")
        w("  const int lane = threadIdx.x;")
        w("  const int64_t ev = (int64_t)blockIdx.x * 64 + lane;")
        w("  const int64_t evc = ev < nev ? ev : nev - 1;")
        w("  double pm[NEXT][4];")
        w("  load_momenta<NEXT>(mom, evc, pm);")
        if not self.reg_jamp:
            w("  __shared__ double2 jl[NCOL][64];")
        w("  double q = 0.0;")
        for i, p in enumerate(self.pats):
            w("#pragma unroll 1")
            w(f"  for (int cfg = 0; cfg < {p.ncfg}; ++cfg) {{")
            w("    double pp[NEXT][4];")
            w("    opaque_copy<NEXT>(pm, pp);")
            call = f"pattern{i}<R>(pp, cfg)" if self.reg_jamp else f"pattern{i}<R>(pp, cfg, jl, lane, cmat)"
            w(f"    q += {call};")
            w("  }")
        w("  if (ev < nev) out[ev] = q * scale;")
        w("}")
        w(f"template __global__ void me2_kernel<double>({kern_args});")
        w(f"template __global__ void me2_kernel<float>({kern_args});")
        w("")
        w(f"}}  // namespace {ns}")
        w("}  // namespace heget")
        w("")
        # host side launcher and descriptor (host compilation pass only)
        w("#if !defined(__HIP_DEVICE_COMPILE__)")
        table = self.colour_table() if not self.reg_jamp else []
        w(f"static const double k_colour_table_{proc.tag}[] = {{" +
          (", ".join(_lit(x) for x in table) if table else "0.0") + "};")
        nvals = []
        for a in range(self.k):
            for b in range(self.k):
                v = self.nmat[a][b]
                nvals.append((v.numerator, v.denominator))
        w(f"static const long long k_num_{proc.tag}[] = {{" + ", ".join(str(x[0]) for x in nvals) + "};")
        w(f"static const long long k_den_{proc.tag}[] = {{" + ", ".join(str(x[1]) for x in nvals) + "};")
        w(f"static hipError_t launch_{proc.tag}(int prec, const double* mom, int64_t n, double* out, "
          f"const double* cmat, double scale, hipStream_t s) {{")
        w("  const dim3 grid((unsigned)((n + 63) / 64)), block(64);")
        w("  if (prec == 0)")
        w(f"    hipLaunchKernelGGL(heget::{ns}::me2_kernel<double>, grid, block, 0, s, mom, n, out, cmat, scale);")
        w("  else")
        w(f"    hipLaunchKernelGGL(heget::{ns}::me2_kernel<float>, grid, block, 0, s, mom, n, out, cmat, scale);")
        w("  return hipGetLastError();")
        w("}")
        nhel = 2 * sum(p.ncfg for p in self.pats)
        w(f"extern const heget_proc_desc heget_desc_{proc.tag} = {{")
        w(f"  \"{proc.spec}\", {proc.n}, {len(dag.amps)}, {self.k}, {nhel}, {1 << proc.n},")
        w(f"  {len(table)}, k_colour_table_{proc.tag}, k_num_{proc.tag}, k_den_{proc.tag},")
        w(f"  {self.flops_per_event}LL, launch_{proc.tag}}};")
        w("#endif")
        return "\n".join(lines) + "\n"
