"""Measured choice of the kernel planner's per-process settings.

    python -m paper_0909_5257_amd.tune build   --out DIR [--only SPEC ...]   # on the build host
    python -m paper_0909_5257_amd.tune measure --out DIR                     # on the GPU
    python -m paper_0909_5257_amd.tune apply   --out DIR                     # writes gen/tuned.py

`build` compiles one library per candidate setting (every listed process built with it), `measure`
times every (process, precision, candidate) on the GPU with HIP events around the |M|^2 launch, each
library in a process of its own, and `apply` keeps, per process and precision, the fastest candidate
when it beats the default by more than the noise margin.  The candidates are the two ways of
handling external wavefunctions (kept in registers across a chunk's groups, or rebuilt inside every
group from the LDS momenta) and the simulated register budget of a group.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# name -> {precision: settings}; "default" is the planner without a table entry
CANDIDATES = {
    "default": {},
    "group208": {"double": {"externals": "group", "budget": 208}, "float": {"externals": "group", "budget": 176}},
    "group256": {"double": {"externals": "group", "budget": 256}, "float": {"externals": "group", "budget": 208}},
    "group320": {"double": {"externals": "group", "budget": 320}, "float": {"externals": "group", "budget": 240}},
    # more resident waves: float64 at two per SIMD, float32 at three
    "group176w": {"double": {"externals": "group", "budget": 176, "waves_per_cu": 8},
                  "float": {"externals": "group", "budget": 144, "waves_per_cu": 12}},
    # externals kept in registers, other budgets
    "keep160": {"double": {"budget": 160}, "float": {"budget": 160}},
    "keep200": {"double": {"budget": 192}, "float": {"budget": 200}},
    "keep224": {"double": {"budget": 224}, "float": {"budget": 224}},
    "keep256": {"double": {"budget": 256}, "float": {"budget": 192}},
    # large float64 groups (the inlined helicity loop leaves the float64 kernels the whole register
    # file), small float32 ones (the float32 kernels spill at two waves per SIMD)
    "keep288": {"double": {"budget": 288}, "float": {"budget": 144}},
    # the same with one call of the wave's work per helicity configuration instead of the loop inlined
    # into the kernel (fewer registers spilled inside the loop where the inlined body spills)
    "keep224c": {"double": {"budget": 224, "calls": True}, "float": {"budget": 224, "calls": True}},
    # one wave per 64-event group where the colour vector is small enough: no cross-wave
    # accumulation, bit-reproducible results
    # float64 budgets around the kept-externals optimum of u u~ > 5g (float: its group-local 208)
    "keep240": {"double": {"budget": 240}, "float": {"externals": "group", "budget": 208}},
    "keep264": {"double": {"budget": 264}, "float": {"externals": "group", "budget": 208}},
    "keep272": {"double": {"budget": 272}, "float": {"externals": "group", "budget": 208}},
    "keep280": {"double": {"budget": 280}, "float": {"externals": "group", "budget": 208}},
    # group-local float32 budgets around 208, with float64 kept-externals budgets around 256
    "g192": {"double": {"budget": 240}, "float": {"externals": "group", "budget": 192}},
    "g224": {"double": {"budget": 272}, "float": {"externals": "group", "budget": 224}},
    "g240": {"double": {"budget": 288}, "float": {"externals": "group", "budget": 240}},
    # two float64 waves per SIMD (eight per 64-event workgroup of u u~ > 5g), registers for 256 each
    "w8k176": {"double": {"budget": 176, "waves_per_cu": 8}, "float": {"externals": "group", "budget": 208}},
    "w8g192": {"double": {"externals": "group", "budget": 192, "waves_per_cu": 8},
               "float": {"externals": "group", "budget": 208}},
    "group176s": {"double": {"externals": "group", "budget": 176},
                  "float": {"externals": "group", "budget": 176, "waves_per_cu": 4}},
}
DEFAULT_PROCESSES = ["g g > g g g g", "u u~ > g g g g", "u u~ > g g g g g", "u u > u u g g", "u u > u u g g g",
                     "u g > u g g g"]
MARGIN = 0.03          # a candidate must be this much faster than the default to be kept
EVENTS = 1 << 18


def _build(args):
    procs = args.only or DEFAULT_PROCESSES
    os.makedirs(args.out, exist_ok=True)
    names = args.candidates or list(CANDIDATES)
    jobs = max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)) // len(names))
    running = []
    for name in names:                          # the candidate builds run side by side
        cand = CANDIDATES[name]
        env = dict(os.environ)
        env["HEGET_GEN_DIR"] = os.path.join(args.out, f"gen_{name}")
        env["HEGET_BUILD_DIR"] = os.path.join(args.out, f"build_{name}")
        env["HEGET_LIB_OUT"] = os.path.join(args.out, f"lib_{name}.so")
        env["HEGET_TUNED_JSON"] = json.dumps({f"{spec}|{prec}": s for spec in procs for prec, s in cand.items()})
        env["HEGET_TUNED_REPLACE"] = "1"
        print(f"[tune] building {name}", flush=True)
        log = open(os.path.join(args.out, f"build_{name}.log"), "w")
        running.append((name, log, subprocess.Popen(
            [sys.executable, "-m", "paper_0909_5257_amd.build", "--jobs", str(jobs), "--only", *procs],
            env=env, cwd=ROOT, stdout=log, stderr=subprocess.STDOUT)))
    for name, log, proc in running:
        if proc.wait() != 0:
            raise SystemExit(f"build of candidate {name} failed (see {log.name})")
        log.close()
        print(f"[tune] built {name}", flush=True)
    with open(os.path.join(args.out, "processes.json"), "w") as f:
        json.dump(procs, f)


_TIMER = r"""
import json, sys
import torch
sys.path.insert(0, ROOT)
from phasespace import KIN_C2, generate_events
from paper_0909_5257_amd.heget import Process
out = {}
for spec in SPECS:
    nf = len(spec.split(">")[1].split())
    p = torch.from_numpy(generate_events(EVENTS, nf, KIN_C2, seed=0)).cuda()
    for prec in ("fp64", "mixed"):
        pr = Process(spec, prec)
        res = pr.matrix_elements(p, 0.118)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            pr.matrix_elements(p, 0.118, out=res)
        b.record()
        torch.cuda.synchronize()
        out[spec + "|" + prec] = a.elapsed_time(b) / 3
        print(spec, prec, out[spec + "|" + prec], flush=True)
print("RESULT " + json.dumps(out), flush=True)
"""


def _measure(args):
    procs = json.load(open(os.path.join(args.out, "processes.json")))
    path = os.path.join(args.out, "timings.json")
    results = json.load(open(path)) if os.path.exists(path) else {}    # earlier candidates are kept
    for name in args.candidates or list(CANDIDATES):
        lib = os.path.join(args.out, f"lib_{name}.so")
        code = _TIMER.replace("ROOT", repr(ROOT)).replace("SPECS", repr(procs)).replace("EVENTS", str(EVENTS))
        env = dict(os.environ, HEGET_LIB=lib)
        print(f"[tune] timing {name}", flush=True)
        run = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        sys.stdout.write(run.stdout)
        if run.returncode != 0:
            sys.stderr.write(run.stderr[-3000:])
            raise SystemExit(f"timing with {name} failed")
        line = [l for l in run.stdout.splitlines() if l.startswith("RESULT ")][-1]
        results.setdefault(name, {}).update(json.loads(line[len("RESULT "):]))
    with open(path, "w") as f:
        json.dump(results, f, indent=1)


def _current_table() -> dict:
    from .gen.tuned import TUNED
    return dict(TUNED)


def _apply(args):
    timings = json.load(open(os.path.join(args.out, "timings.json")))
    # settings of processes this run did not time stay as they are
    timed = {k.split("|")[0] for k in timings["default"]}
    chosen = {key: val for key, val in _current_table().items() if key[0] not in timed}
    keys = sorted(timings["default"])
    for key in keys:
        spec, prec = key.split("|")
        gprec = "double" if prec == "fp64" else "float"
        base = timings["default"][key]
        best, best_ms = None, base
        for name, t in timings.items():
            if name != "default" and key in t and t[key] < best_ms:
                best, best_ms = name, t[key]
        print(f"{key:28s} default {base:9.2f} ms  best {best or 'default':9s} {best_ms:9.2f} ms", flush=True)
        if best is not None and best_ms < (1.0 - MARGIN) * base:
            chosen[(spec, gprec)] = dict(CANDIDATES[best][gprec], ms=round(best_ms, 3), default_ms=round(base, 3))
    lines = ['"""Per-process planner settings chosen by measurement (python -m paper_0909_5257_amd.tune).',
             "",
             f"Timed on one MI355X: {EVENTS} events per launch, seeded RAMBO events with sqrt(s) U[300, 2000]",
             'GeV and the jet cuts; ms = mean of three launches with the setting, default_ms = without it."""',
             "", "TUNED = {"]
    for (spec, gprec), s in sorted(chosen.items()):
        lines.append(f"    ({spec!r}, {gprec!r}): {s!r},")
    lines.append("}")
    table = args.table or os.path.join(HERE, "gen", "tuned.py")
    with open(table, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"[tune] wrote {len(chosen)} settings to {table}", flush=True)
    return chosen


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("step", choices=["build", "measure", "apply"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--only", nargs="*")
    ap.add_argument("--table", default=None, help="output of apply (default: gen/tuned.py)")
    ap.add_argument("--candidates", nargs="*", help="build / time only these candidates")
    args = ap.parse_args(argv)
    return {"build": _build, "measure": _measure, "apply": _apply}[args.step](args)


if __name__ == "__main__":
    main()
