"""Generate the per-process HIP kernels and build libheget.so for gfx950.

    python -m paper_0909_5257_amd.build [--only TAG ...] [--jobs N] [--resource-usage]

Steps: for every supported process, build the shared-current DAG and the
exact colour matrix, emit csrc/generated/proc_<tag>_{f64,f32}.hip and a registry, then
compile each translation unit with hipcc for gfx950 and link the shared
library next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN_DIR = os.environ.get("HEGET_GEN_DIR", os.path.join(CSRC, "generated"))
BUILD_DIR = os.environ.get("HEGET_BUILD_DIR", os.path.join(ROOT, "_build"))
LIB = os.environ.get("HEGET_LIB_OUT", os.path.join(HERE, "libheget.so"))

# The processes of the paper's Table 1 whose kernels are compiled in.
PROCESSES = [
    "g g > g g", "g g > g g g", "g g > g g g g",
    # 7,245 diagrams, 720 colours: the paper could not compile it for its GPU
    "g g > g g g g g",
    "u u~ > g g", "u u~ > g g g", "u u~ > g g g g", "u u~ > g g g g g",
    "u u > u u", "u u > u u g", "u u > u u g g", "u u > u u g g g",
    # crossed subprocesses: same diagram and colour counts as u u~ > n g
    "u g > u g", "u g > u g g", "u g > u g g g",
    "u u~ > u u~",
]

# processes with at most this many legs also get the test-hook kernels (gauge substitution and
# colour-vector export, include/heget.h heget_matrix_elements_hook)
HOOK_MAX_LEGS = 6

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
]
# tuning knobs of the kernel planner, overridable from the environment (HEGET_<NAME>); the
# per-precision ones take "float64_value,float32_value"
for _name in ("CHUNK_FLOPS", "COOP_CHUNK_FLOPS", "TARGET_WAVES_PER_CU", "FORCE_WAVES",
              "MERGE_WAVE_CHUNKS", "MERGE_MAX_PATTERN_FLOPS"):
    if os.environ.get("HEGET_" + _name):
        from .gen import emit as _emit
        _val = os.environ["HEGET_" + _name]
        if isinstance(getattr(_emit, _name), dict):
            _d, _f = (int(x) for x in _val.split(","))
            setattr(_emit, _name, {"double": _d, "float": _f})
        else:
            setattr(_emit, _name, int(_val))
if os.environ.get("HEGET_TUNED_JSON"):
    # planner settings per "process|double|float" key, from the tuner; HEGET_TUNED_REPLACE=1 drops
    # the committed table first (so that the tuner's default candidate really is the default)
    import json as _json
    from .gen import emit as _emit
    _extra = {tuple(k.split("|")): v for k, v in _json.loads(os.environ["HEGET_TUNED_JSON"]).items()}
    if os.environ.get("HEGET_TUNED_REPLACE") == "1":
        _emit.TUNED = {}
    _emit.TUNED.update(_extra)
for _prec in ("double", "float"):
    _env = os.environ.get(f"HEGET_GROUP_BUDGET_{'F64' if _prec == 'double' else 'F32'}")
    if _env:
        from .gen import emit as _emit
        _emit.GROUP_BUDGET[_prec] = int(_env)


def generate(specs, verbose=True):
    from .gen.emit import Emitter
    from .gen.model import Dag, parse

    os.makedirs(GEN_DIR, exist_ok=True)
    files, tags = [], []
    for spec in specs:
        t0 = time.time()
        dag = Dag(parse(spec))
        nmat = dag.colour_matrix()
        hook = dag.proc.n <= HOOK_MAX_LEGS
        srcs = Emitter(dag, nmat).emit(with_hook=hook)
        if hook:
            srcs["hook"] = Emitter(dag, nmat, hook=True).emit_hook()
        for part, src in srcs.items():
            path = os.path.join(GEN_DIR, f"proc_{dag.proc.tag}_{part}.hip")
            _write_if_changed(path, src)
            files.append(path)
        tags.append(dag.proc.tag)
        if verbose:
            print(f"[gen] {spec:22s} -> proc_{dag.proc.tag}_{{{','.join(srcs)}}}.hip ({time.time() - t0:.1f}s)",
                  flush=True)
    # drop generated sources of processes (or layouts) this build does not contain
    for name in os.listdir(GEN_DIR):
        path = os.path.join(GEN_DIR, name)
        if name.startswith("proc_") and name.endswith(".hip") and path not in files:
            os.remove(path)
    reg = ['#include "heget_kernel_common.hpp"']
    reg += [f"extern const heget_proc_desc heget_desc_{t};" for t in tags]
    reg.append("extern const heget_proc_desc* const heget_registry[] = {")
    reg += [f"  &heget_desc_{t}," for t in tags]
    reg.append("};")
    reg.append(f"extern const int heget_registry_len = {len(tags)};")
    reg_path = os.path.join(GEN_DIR, "registry.cpp")
    _write_if_changed(reg_path, "\n".join(reg) + "\n")
    return files, reg_path


def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, "w") as f:
        f.write(text)


def _local_includes(path, seen):
    """path and every file it includes with #include "..." from csrc/ or include/, recursively."""
    if path in seen:
        return
    seen.append(path)
    for line in open(path, errors="replace"):
        line = line.strip()
        if line.startswith("#include \""):
            name = line.split('"')[1]
            for d in (CSRC, os.path.join(ROOT, "include")):
                cand = os.path.join(d, name)
                if os.path.exists(cand):
                    _local_includes(cand, seen)
                    break


def _digest(src, cmd):
    """Digest of the command, the source and the local headers it includes (so that editing the
    public header does not recompile the generated process units, which never include it)."""
    h = hashlib.sha256(" ".join(cmd).encode())
    files = []
    _local_includes(src, files)
    for path in files:
        h.update(path.encode())
        h.update(open(path, "rb").read())
    return h.hexdigest()


def _compile(src, extra, force=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC] + FLAGS + extra + lang + ["-c", src, "-o", obj]
    stamp = obj + ".sha"
    digest = _digest(src, cmd)
    if not force and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == digest:
        return obj, 0.0, ""
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stderr[-4000:]}")
    with open(stamp, "w") as f:
        f.write(digest)
    return obj, time.time() - t0, res.stderr


def build(specs=None, jobs=None, resource_usage=False, verbose=True, force=False):
    specs = specs or PROCESSES
    files, reg = generate(specs, verbose)
    srcs = [os.path.join(CSRC, "heget.cpp"), os.path.join(CSRC, "colour_gemm.cpp"),
            os.path.join(CSRC, "phase_space.cpp"), reg] + files
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    objs = []
    srcs = sorted(srcs, key=lambda p: -os.path.getsize(p))      # longest compiles start first
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = {ex.submit(_compile, s, extra, force): s for s in srcs}
        for fut in cf.as_completed(futs):
            obj, dt, log = fut.result()
            objs.append(obj)
            if verbose:
                print(f"[hipcc] {os.path.basename(futs[fut]):32s} {dt:6.1f}s", flush=True)
            if resource_usage and log:
                print(log, flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + sorted(objs) + \
        ["-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {res.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[link] {LIB}", flush=True)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", help="process specs to build (default: all)")
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--resource-usage", action="store_true")
    ap.add_argument("--force", action="store_true", help="recompile even when sources are unchanged")
    a = ap.parse_args(argv)
    build(a.only, a.jobs, a.resource_usage, force=a.force)


if __name__ == "__main__":
    main()
