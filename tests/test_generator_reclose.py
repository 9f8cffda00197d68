"""The generator's choice of closing vertex (Dag._reclose) leaves every diagram's amplitude unchanged.

A diagram's amplitude does not depend on the vertex at which its currents are finally contracted;
the generator moves the contraction next to the root where that saves a current.  This test
evaluates every diagram of both DAGs (root closure and reclosed) with a numpy transcription of the
device routines (the formulas of paper_0909_5257_amd/csrc/heget_device.hpp: polarisation
vectors, two-component spinors, the three- and four-gluon and quark-gluon vertices and currents)
on seeded events and helicity configurations, and requires equality to rounding.  It checks the
rewrite only: the routines themselves are checked against the oracle by the GPU parity tests.
The same transcription checks the emitter's merged closing vertices (one contraction with summed
operands for the diagrams of a colour class that differ in one operand).
"""
import numpy as np
import pytest

from phasespace import KIN_C2, generate_events


def _mdot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def _pol(p, lam, outgoing):
    pt = np.hypot(p[1], p[2])
    pa = np.sqrt(pt * pt + p[3] * p[3])
    ct, st = p[3] / pa, pt / pa
    cf, sf = (p[1] / pt, p[2] / pt) if pt > 0 else (1.0, 0.0)
    l = np.sqrt(0.5) * (1 if lam > 0 else -1)
    im = -np.sqrt(0.5) if outgoing else np.sqrt(0.5)
    return np.array([0, -l * ct * cf + 1j * im * sf, -l * ct * sf - 1j * im * cf, l * st], complex)


def _xi(p, h):
    rho = p[0] + p[3]
    if rho > 1e-10 * p[0]:
        sr = np.sqrt(rho)
        return np.array([sr, (p[1] + 1j * p[2]) / sr]) if h > 0 else np.array([(-p[1] + 1j * p[2]) / sr, sr])
    s2 = np.sqrt(2 * p[0])
    return np.array([0, s2], complex) if h > 0 else np.array([-s2, 0], complex)


def _smat(v, h):
    return np.array([[v[0] - h * v[3], -h * (v[1] - 1j * v[2])], [-h * (v[1] + 1j * v[2]), v[0] + h * v[3]]])


def _vvv(a, pa, b, pb, c, pc):
    return -(_mdot(a, b) * _mdot(pa - pb, c) + _mdot(b, c) * _mdot(pb - pc, a) + _mdot(c, a) * _mdot(pc - pa, b))


def _gggg(a, b, c, d):
    return _mdot(a, d) * _mdot(b, c) - _mdot(a, c) * _mdot(b, d)


def _closing(dag, amp, a, pm, w, pw, hq):
    """The closing vertex of one diagram for operand values a with momenta pm (root value w, pw)."""
    h = hq.get(dag.nodes[amp.args[0]].end)
    if amp.op == "vvv":
        return _vvv(a[0], pm[0], a[1], pm[1], w, pw)
    if amp.op == "gggg":
        x, y, z = a
        return _gggg(*[(x, y, z, w), (x, z, w, y), (x, w, y, z)][amp.piece])
    if amp.op == "iov":
        return w @ (_smat(a[1], h) @ a[0])
    if amp.op == "vvvx":
        return _vvv(a[0], pm[0], a[1], pm[1], a[2], pm[2])
    if amp.op == "ggggx":
        return _gggg(*a)
    return a[1] @ (_smat(a[2], h) @ a[0])


def _amplitudes(dag, pmom, lam, hq, with_values=False):
    proc, nd = dag.proc, dag.nodes

    def mom(mask):
        return sum((-pmom[i] if proc.legs[i].incoming else pmom[i]) for i in range(proc.n) if mask >> i & 1)
    val = {}
    for n in nd:
        if n.op == "ext":
            leg, p = proc.legs[n.leg], pmom[n.leg]
            if leg.kind == "V":
                val[n.id] = _pol(p, lam[n.leg], not leg.incoming)
            else:
                x = _xi(p, hq[n.leg]).astype(complex)
                val[n.id] = x if leg.kind == "I" else np.conj(x)
            continue
        a = [val[x] for x in n.args]
        pm = [mom(nd[x].mask) for x in n.args]
        inv = 1.0 / _mdot(mom(n.mask), mom(n.mask)).real
        if n.op == "jvv":
            sa, sb = pm[0] + 2 * pm[1], 2 * pm[0] + pm[1]
            val[n.id] = inv * (-(pm[0] - pm[1]) * _mdot(a[0], a[1]) - _mdot(sa, a[0]) * a[1] + _mdot(sb, a[1]) * a[0])
        elif n.op == "jggg":
            val[n.id] = inv * (_mdot(a[2], a[1]) * a[0] - _mdot(a[0], a[2]) * a[1])
        elif n.op == "jio":
            fi, fo, h = a[0], a[1], hq[nd[n.args[0]].end]
            val[n.id] = inv * np.array([fo[0] * fi[0] + fo[1] * fi[1], h * (fo[0] * fi[1] + fo[1] * fi[0]),
                                        h * 1j * (fo[1] * fi[0] - fo[0] * fi[1]), h * (fo[0] * fi[0] - fo[1] * fi[1])])
        elif n.op == "fvi":
            h = hq[n.end]
            val[n.id] = inv * (_smat(mom(n.mask), -h) @ (_smat(a[1], h) @ a[0]))
        elif n.op == "fvo":
            h = hq[n.end]
            val[n.id] = -inv * ((a[0] @ _smat(a[1], h)) @ _smat(mom(n.mask), -h))
    root = proc.root
    w, pw = val[dag.ext[root]], mom(1 << root)
    out = []
    for amp in dag.amps:
        out.append(_closing(dag, amp, [val[x] for x in amp.args], [mom(nd[x].mask) for x in amp.args], w, pw, hq))
    if with_values:
        return np.array(out), val, mom
    return np.array(out)


@pytest.mark.parametrize("spec", ["g g > g g", "g g > g g g", "g g > g g g g", "u u~ > g g", "u u~ > g g g",
                                  "u u~ > g g g g", "u g > u g g", "u u > u u g", "u u > u u g g", "u u~ > u u~"])
def test_reclosed_amplitudes_equal_root_closed(spec, monkeypatch):
    from paper_0909_5257_amd.gen import model
    from paper_0909_5257_amd.gen.emit import Emitter
    monkeypatch.setattr(model, "RECLOSE", False)
    d0 = model.Dag(model.parse(spec))
    monkeypatch.setattr(model, "RECLOSE", True)
    d1 = model.Dag(model.parse(spec))
    assert len(d1.amps) == len(d0.amps) and len(d1.nodes) <= len(d0.nodes)
    assert [a.coef for a in d1.amps] == [a.coef for a in d0.amps]          # same diagrams, same colour
    em = Emitter(d1, d1.colour_matrix())
    ev = generate_events(3, d1.proc.n - 2, KIN_C2, seed=5)
    worst = 0.0
    for pat in em.pats:
        for cfg in range(min(pat.ncfg, 8)):
            lam = {0: 1, **{g: (1 if (cfg >> j) & 1 else -1) for j, g in enumerate(pat.free_gluons)}, **pat.fixed}
            for q, h in pat.hq.items():
                lam[q] = h if d1.proc.legs[q].flavour == "u" else -h
            for p in ev:
                a0 = _amplitudes(d0, p, lam, pat.hq)[pat.amps]
                a1 = _amplitudes(d1, p, lam, pat.hq)[pat.amps]
                worst = max(worst, np.abs(a1 - a0).max() / np.abs(a0).max())
    assert worst < 1e-12


@pytest.mark.parametrize("spec,any_merge", [("g g > g g g g", True), ("u u~ > g g g g", True),
                                            ("u u > u u g g", False), ("u g > u g g", False), ("u u~ > u u~", False)])
def test_merged_closing_vertices_equal_diagram_sums(spec, any_merge):
    """The emitter's merge plan: within a colour class, diagrams that differ only in one operand of
    their closing vertex (same external legs, hence the same momentum) are contracted once with the
    summed operand.  By linearity of every vertex in each operand, fac_0 V(..., sum_i fac_i/fac_0 X_i,
    ...) equals sum_i fac_i V(..., X_i, ...); the plan covers each amplitude of the class once."""
    from fractions import Fraction
    from paper_0909_5257_amd.gen.emit import Emitter, colour_classes
    from paper_0909_5257_amd.gen.model import Dag, parse
    dag = Dag(parse(spec))
    em = Emitter(dag, dag.colour_matrix())
    nd = dag.nodes
    ev = generate_events(2, dag.proc.n - 2, KIN_C2, seed=6)
    worst, merged = 0.0, 0
    for pat in em.pats:
        lam = {0: 1, **{g: (1 if j % 2 else -1) for j, g in enumerate(pat.free_gluons)}, **pat.fixed}
        for q, h in pat.hq.items():
            lam[q] = h if dag.proc.legs[q].flavour == "u" else -h
        for p in ev:
            amps, val, mom = _amplitudes(dag, p, lam, pat.hq, with_values=True)
            w, pw = val[dag.ext[dag.proc.root]], mom(1 << dag.proc.root)
            for _, members in colour_classes(em.vectors, pat.amps):
                plan = em.merge_plan(members)
                covered = sorted(ai for kind, d in plan for ai in ([d[0]] if kind == "one" else [x for x, _ in d[1]]))
                assert covered == sorted(ai for ai, _ in members)
                for kind, d in plan:
                    if kind == "one":
                        continue
                    pos, grp = d
                    a0, f0 = grp[0]
                    amp0 = dag.amps[a0]
                    for ai, _ in grp:
                        other = dag.amps[ai]
                        assert other.op == amp0.op and other.piece == amp0.piece
                        assert all(x == y for q, (x, y) in enumerate(zip(other.args, amp0.args)) if q != pos)
                        assert nd[other.args[pos]].mask == nd[amp0.args[pos]].mask
                    direct = sum(float(f) * amps[ai] for ai, f in grp)
                    xsum = sum(float(Fraction(f) / Fraction(f0)) * val[dag.amps[ai].args[pos]] for ai, f in grp)
                    a = [xsum if q == pos else val[x] for q, x in enumerate(amp0.args)]
                    once = float(f0) * _closing(dag, amp0, a, [mom(nd[x].mask) for x in amp0.args], w, pw, pat.hq)
                    worst = max(worst, abs(once - direct) / max(abs(amps[pat.amps]).max(), 1e-300))
                    merged += 1
    assert (merged > 0) == any_merge and worst < 1e-12
