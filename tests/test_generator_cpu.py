"""Host-side checks of the process generator and of the built C ABI (no GPU needed)."""
import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from paper_0909_5257_amd.gen import colour_algebra as ca
from paper_0909_5257_amd.gen.emit import Emitter, colour_classes, patterns
from paper_0909_5257_amd.gen.model import Dag, parse

from conftest import ROOT, golden

SMALL = ["g g > g g", "g g > g g g", "u u~ > g g", "u u~ > g g g", "u u~ > g g g g",
         "u u > u u", "u u > u u g", "u u > u u g g"]


def _table(name):
    rows = []
    for line in open(golden(name)):
        if line.strip() and not line.startswith("#"):
            rows.append([x.strip() for x in line.split("|")])
    return rows


@pytest.mark.parametrize("row", _table("paper_table1.txt"), ids=lambda r: r[0])
def test_generator_table1(row):
    dag = Dag(parse(row[0]))
    assert len(dag.amps) == int(row[1])
    assert len(dag.basis) == int(row[2])


@pytest.mark.parametrize("row", [r for r in _table("paper_table3.txt") if r[0] in SMALL + ["g g > g g g g g"]],
                         ids=lambda r: r[0])
def test_generator_table3(row):
    dag = Dag(parse(row[0]))
    n = dag.colour_matrix()
    vals = {n[i][j] for i in range(len(n)) for j in range(i, len(n))} - {Fraction(0)}
    assert len(vals) == int(row[1])


@pytest.mark.parametrize("spec", SMALL)
def test_generator_colour_matrix_equals_oracle(spec):
    """The generator's Fierz-reduced N equals the oracle's literal colour sum exactly."""
    from oracle.colour import colour_data
    dag = Dag(parse(spec))
    n = dag.colour_matrix()
    cd = colour_data(spec)
    assert n == cd.N_frac


@pytest.mark.parametrize("spec,n_hel", [("g g > g g", 16), ("g g > g g g g", 64), ("u u~ > g g g", 16),
                                        ("u u~ > g g g g g", 64), ("u u > u u", 6), ("u u > u u g g", 24)])
def test_helicity_patterns(spec, n_hel):
    """Evaluated configurations x 2 (flip partner) = non-zero helicity configurations."""
    dag = Dag(parse(spec))
    assert 2 * sum(p.ncfg for p in patterns(dag)) == n_hel


def test_every_diagram_has_a_colour_class():
    dag = Dag(parse("g g > g g g g"))
    amps = list(range(len(dag.amps)))
    classes = colour_classes({i: a.coef for i, a in enumerate(dag.amps)}, amps)
    assert sum(len(m) for _, m in classes) == len(amps)
    # every cubic tree of 6 gluons is its own class: (2*6-5)!! = 105
    assert len(classes) == 105


def test_fierz_reduction_basics():
    # Tr(T^a T^a) = C_F N = 4, Tr(T^a) Tr(T^a) = 0, Tr(T^a T^b T^a T^b) = -2/3
    assert ca._reduce(ca._canon([(0, 0)])) == 4
    assert ca._reduce(ca._canon([(0,), (0,)])) == 0
    assert ca._reduce(ca._canon([(0, 1, 0, 1)])) == Fraction(-2, 3)


def test_colour_commutator_matches_structure_constants():
    """[T^a, T^b] expansions give the two orderings with opposite signs."""
    m = ca.comm(ca.Poly.letter(1), ca.Poly.letter(2))
    assert m.terms == {((), (1, 2)): (1, 0), ((), (2, 1)): (-1, 0)}


# ------------------------------------------------------------ built library

def _header_functions():
    text = open(os.path.join(ROOT, "include", "heget.h")).read()
    return sorted(set(re.findall(r"\b(heget_[a-z_]+)\s*\(", text)))


def test_library_exports_header_symbols():
    path = os.path.join(ROOT, "paper_0909_5257_amd", "libheget.so")
    if not os.path.exists(path):
        pytest.skip("libheget.so not built (python -m paper_0909_5257_amd.build)")
    lib = ctypes.CDLL(path)
    names = _header_functions()
    assert "heget_matrix_elements" in names and "heget_create_process" in names
    for name in names:
        assert hasattr(lib, name), name


def test_library_registry_and_status_strings():
    path = os.path.join(ROOT, "paper_0909_5257_amd", "libheget.so")
    if not os.path.exists(path):
        pytest.skip("libheget.so not built")
    from paper_0909_5257_amd import heget
    specs = heget.supported_processes()
    assert "g g > g g" in specs
    L = heget.lib()
    assert L.heget_status_string(0) == b"ok"
    assert L.heget_process_spec(-1) is None
    # argument errors are reported before any device call
    h = ctypes.c_void_p()
    assert L.heget_create_process(None, 0, ctypes.byref(h)) == 1
    assert L.heget_create_process(b"g g > g g", 7, ctypes.byref(h)) == 1
    assert L.heget_matrix_elements(None, None, 0, 0.118, None, None) == 1


@pytest.mark.parametrize("spec", ["g g > g g g", "g g > g g g g", "u u~ > g g g g", "u u > u u g", "u u > u u g g"])
def test_reduced_colour_space_is_exact(spec):
    """y^H W y in the reduced space equals J^H N J in the paper's basis for arbitrary amplitudes."""
    from paper_0909_5257_amd.gen.reduce import ColourSpace
    dag = Dag(parse(spec))
    nmat = dag.colour_matrix()
    cs = ColourSpace(dag, nmat)
    rng = np.random.default_rng(5)
    k = len(dag.basis)
    nf = np.array([[float(x) for x in r] for r in nmat])
    w = np.array([[float(x) for x in r] for r in cs.w])
    for _ in range(3):
        amp = rng.normal(size=len(dag.amps)) + 1j * rng.normal(size=len(dag.amps))
        jv = np.zeros(k, complex)
        yv = np.zeros(cs.dim, complex)
        for i, a in enumerate(dag.amps):
            for idx, v in a.coef.items():
                jv[idx] += v * amp[i]
            for idx, v in cs.vector(a.coef).items():
                yv[idx] += float(v) * amp[i]
        q_full = (jv @ nf @ jv.conj()).real
        q_red = (yv @ w @ yv.conj()).real
        assert abs(q_red / q_full - 1) < 1e-13
    assert cs.dim <= k


@pytest.mark.parametrize("spec", ["g g > g g g", "u u~ > g g g", "u u > u u g", "u g > u g g", "u u~ > u u~"])
def test_helicity_map_covers_each_configuration_once(spec):
    """The sampled-helicity table reaches every evaluated configuration from exactly one
    leg-0-positive pattern, and its structural zeros are those of the oracle."""
    from oracle import oracle_me2
    from phasespace import KIN_C2, generate_events
    dag = Dag(parse(spec))
    em = Emitter(dag, dag.colour_matrix())
    hmap = em.helicity_map()
    n = dag.proc.n
    codes = [hmap[h] for h in range(1 << n) if h & 1 and hmap[h] >= 0]
    assert len(codes) == len(set(codes)) == sum(p.ncfg for p in em.pats)
    p = generate_events(3, n - 2, KIN_C2, seed=4)
    _, per_hel = oracle_me2(spec, p, 0.118, return_helicities=True)
    for h in range(1 << n):
        hp = h if h & 1 else ~h & ((1 << n) - 1)
        # chirality zeros vanish identically in the oracle too (dynamic zeros such as
        # all-but-one equal gluon helicities only to rounding, and are evaluated)
        oracle_zero = bool(np.all(per_hel[h] == 0.0))
        assert (hmap[hp] < 0) == oracle_zero, h


@pytest.mark.parametrize("spec", ["g g > g g g", "g g > g g g g", "u u~ > g g g g", "u u > u u g g g"])
def test_workgroup_shape_fits_lds_and_meets_occupancy_target(spec):
    """Every kernel's static LDS fits one CU and the chosen waves per workgroup reach the
    precision's resident-wave target (or the largest shape is taken)."""
    from paper_0909_5257_amd.gen import emit
    dag = Dag(parse(spec))
    em = Emitter(dag, dag.colour_matrix())
    for prec in ("double", "float"):
        w = em.nwave[prec]
        lds = em.lds_bytes(w)
        assert lds <= emit.LDS_PER_CU
        per_cu = emit.LDS_PER_CU // lds
        target = em.target_waves[prec]           # the default, or the tuned value for this process
        assert w * per_cu >= target or w == 8
        if w > 1:       # no smaller shape would have done
            half = w // 2
            assert half * (emit.LDS_PER_CU // em.lds_bytes(half)) < target
    assert em.kdim % em.cblock == 0


def test_tuner_keeps_only_clear_wins(tmp_path):
    """apply keeps, per process and precision, the fastest candidate only when it beats the
    default by more than the margin, and writes a table the planner can read."""
    import json
    import runpy
    from paper_0909_5257_amd import tune
    timings = {
        "default": {"g g > g g g|fp64": 10.0, "g g > g g g|mixed": 10.0},
        "group208": {"g g > g g g|fp64": 9.0, "g g > g g g|mixed": 9.9},
        "group256": {"g g > g g g|fp64": 9.5, "g g > g g g|mixed": 11.0},
        "group320": {"g g > g g g|fp64": 12.0, "g g > g g g|mixed": 12.0},
    }
    (tmp_path / "timings.json").write_text(json.dumps(timings))
    table = tmp_path / "tuned.py"
    chosen = tune.main(["apply", "--out", str(tmp_path), "--table", str(table)])
    # 1 % on mixed is within the margin
    assert {key for key in chosen if key[0] == "g g > g g g"} == {("g g > g g g", "double")}
    from paper_0909_5257_amd.gen.tuned import TUNED
    # settings of processes that were not timed are kept as they are
    assert all(chosen[key] == val for key, val in TUNED.items() if key[0] != "g g > g g g")
    assert chosen[("g g > g g g", "double")]["budget"] == tune.CANDIDATES["group208"]["double"]["budget"]
    loaded = runpy.run_path(str(table))["TUNED"]
    assert loaded[("g g > g g g", "double")]["externals"] == "group"


def test_committed_tuned_table_is_valid():
    from paper_0909_5257_amd.build import PROCESSES
    from paper_0909_5257_amd.gen.tuned import TUNED
    for (spec, prec), s in TUNED.items():
        assert spec in PROCESSES and prec in ("double", "float")
        assert s.get("externals") in (None, "group") and 64 <= s.get("budget", 176) <= 512
        assert s.get("calls") in (None, True)


def _functions(src):
    """(qualifier, name, body) of every device function and kernel in a generated source."""
    out = []
    for m in re.finditer(r"^(__device__ __noinline__|__device__ __forceinline__|__global__[^\n]*?) "
                         r"(?:void|double) (\w+)\([^\n]*\) \{$", src, re.M):
        end = src.index("\n}\n", m.end())
        out.append((m.group(1), m.group(2), src[m.end():end]))
    return out


@pytest.mark.parametrize("spec", ["g g > g g g g", "u u > u u g", "u u~ > g g g g"])
def test_called_functions_hold_no_loop(spec):
    """Generated code structure: the helicity loop of the summed kernel lives in the kernel.  No
    called (noinline) function contains a loop, so no called function needs the long branches
    around a body of several hundred KB that have been compiled with the return-address registers
    as scratch; where a wave's work is one function the summed kernel inlines it."""
    dag = Dag(parse(spec))
    srcs = Emitter(dag, dag.colour_matrix()).emit(with_hook=True)
    srcs["hook"] = Emitter(dag, dag.colour_matrix(), hook=True).emit_hook()
    for part, src in srcs.items():
        src = src if isinstance(src, str) else "\n".join(src)
        fns = _functions(src)
        called = [b for q, n, b in fns if q == "__device__ __noinline__"]
        assert called
        assert not any(re.search(r"\b(for|while)\s*\(", b) for b in called)
        if part != "hook":
            me2 = [b for q, n, b in fns if n.startswith("me2_")]
            assert len(me2) == 1 and "#pragma unroll 1\n    for (int cfg" in me2[0]
            assert not any(re.search(rf"\b{n}\(", me2[0]) for q, n, b in fns if q == "__device__ __noinline__")


@pytest.mark.parametrize("spec", ["g g > g g g", "g g > g g g g", "u u~ > g g g g", "u u > u u g", "u u > u u g g",
                                  "u u~ > u u~"])
def test_reduction_map_and_slot_table(spec):
    """The exported map of the test hooks: the reduced vector the kernels accumulate is exactly
    y = M J for any diagram amplitudes, and the slot table lists each evaluated helicity
    configuration once, in the order the helicity map gives them."""
    dag = Dag(parse(spec))
    em = Emitter(dag, dag.colour_matrix())
    m = np.array([[float(x) for x in row] for row in em.reduction_matrix()])
    rng = np.random.default_rng(8)
    k = len(dag.basis)
    amp = rng.normal(size=len(dag.amps)) + 1j * rng.normal(size=len(dag.amps))
    jv = np.zeros(k, complex)
    yv = np.zeros(em.kdim, complex)
    for i, a in enumerate(dag.amps):
        for idx, v in a.coef.items():
            jv[idx] += v * amp[i]
        for idx, v in em.cs.vector(a.coef).items():
            yv[idx] += float(v) * amp[i]
    assert np.allclose(m @ jv, yv, rtol=0, atol=1e-12 * np.abs(yv).max())
    slots = em.slot_helicities()
    hmap = em.helicity_map()
    assert len(slots) == len(set(slots)) == sum(p.ncfg for p in em.pats)
    offsets = np.cumsum([0] + [p.ncfg for p in em.pats])
    for s, h in enumerate(slots):
        assert h & 1                                  # leg 0 at +1
        pi = int(np.searchsorted(offsets, s, side="right") - 1)
        assert hmap[h] == (pi << 16) | (s - offsets[pi])


@pytest.mark.parametrize("spec", ["g g > g g g g", "u u~ > g g g g", "u u > u u g g", "u g > u g g g"])
def test_greedy_plan_covers_every_amplitude_once(spec):
    """The register plan: every active amplitude of a pattern lands in exactly one group, each colour
    class stays within one group, and a group exceeds the register budget only if it holds a single
    class (a class is never split)."""
    from paper_0909_5257_amd.gen import emit as E
    dag = Dag(parse(spec))
    em = Emitter(dag, dag.colour_matrix())
    for pat in em.pats:
        for prec in ("double", "float"):
            classes, groups = em._plan(pat, prec)
            items = [it for g in groups for it in g]
            assert sorted(ai for _, ai, _ in items) == sorted(pat.amps)
            home = {}
            for gi, g in enumerate(groups):
                for ci, _, _ in g:
                    assert home.setdefault(ci, gi) == gi
                built = E._Group(em, pat, prec, 0)
                for _, ai, fac in g:
                    built.amplitude(ai, "acc", fac)
                assert built.peak() <= em.budget[prec] or len({ci for ci, _, _ in g}) == 1


@pytest.mark.parametrize("spec", ["u u~ > g g g g g", "u u > u u g g g"])
def test_wave_assignment_never_worse_than_longest_first(spec, monkeypatch):
    """Cooperative kernels: the chunk-to-wave assignment after the move/swap refinement has a largest
    wave load no larger than the longest-first assignment's, and it is used only where it gains more
    than REBALANCE_MIN."""
    from paper_0909_5257_amd.gen import emit
    dag = Dag(parse(spec))
    nmat = dag.colour_matrix()
    monkeypatch.setattr(emit, "REBALANCE_MIN", 1.0)             # refinement never kept: plain LPT
    lpt = Emitter(dag, nmat)
    lpt.emit()
    monkeypatch.setattr(emit, "REBALANCE_MIN", 0.02)
    ref = Emitter(dag, nmat)
    ref.emit()
    for prec in ("double", "float"):
        for a, b in zip(lpt.stats[prec], ref.stats[prec]):
            assert sum(a["wave_flops"]) == sum(b["wave_flops"])
            assert max(b["wave_flops"]) <= max(a["wave_flops"])
            assert b["wave_flops"] == a["wave_flops"] or max(b["wave_flops"]) < 0.98 * max(a["wave_flops"])
