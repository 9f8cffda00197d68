"""Write the stored oracle values the GPU parity tests compare against.

    python tests/golden/make_oracle_samples.py [--only NAME ...] [--workers N]

For every sample set below, the seeded synthetic events of a workload are drawn
with phasespace.generate_events (the same call the tests and the benchmark
make), a seeded subset of event indices is chosen, and the FP64 oracle
(oracle.oracle_me2, or the Berends-Giele route oracle.berends_giele.bg_me2 for
seven gluons) evaluates |M|^2 on those events.  Each set is written to
tests/golden/oracle_<name>.txt: a header with the workload parameters and the
SHA-256 of the sampled momenta (so a test can check that it regenerated the
very same events), then one line "index value" per sampled event.

Only oracle/ and phasespace/ (seeded inputs, no matrix-element arithmetic) are
called here; nothing comes from the HIP library.
"""
from __future__ import annotations

import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ALPHA_S = 0.118

# name: (spec, kinematics, n_events, seed, stream, n_sample, index seed)
SETS = {
    # the workload sizes of the parity and benchmark configurations (C1, C2, C3, metric)
    "gg_gg_c1_65536": ("g g > g g", "C1", 65536, 0, 0, 512, 1),
    "uux_gggg_c2_2e20": ("u u~ > g g g g", "C2", 1 << 20, 0, 0, 512, 1),
    "uu_uugg_c2_2e20": ("u u > u u g g", "C2", 1 << 20, 0, 1, 512, 1),
    "gg_gggg_c2_2e21": ("g g > g g g g", "C2", 1 << 21, 0, 1, 512, 1),
    "uux_ggggg_c2_2e20": ("u u~ > g g g g g", "C2", 1 << 20, 0, 0, 512, 1),
    "uu_uuggg_c2_2e18": ("u u > u u g g g", "C2", 1 << 18, 0, 2, 512, 1),
    "gg_ggggg_c2_2e18": ("g g > g g g g g", "C2", 1 << 18, 0, 5, 64, 1),
    # the serving workload's kinematics (C5: sqrt(s) up to 3 TeV), the pools the serving run draws from
    "gg_ggg_c5_2e18": ("g g > g g g", "C5", 1 << 18, 11, 0, 512, 2),
    "gg_gggg_c5_2e18": ("g g > g g g g", "C5", 1 << 18, 11, 1, 512, 2),
    "uux_ggggg_c5_2e18": ("u u~ > g g g g g", "C5", 1 << 18, 11, 2, 512, 2),
    "uu_uuggg_c5_2e18": ("u u > u u g g g", "C5", 1 << 18, 11, 3, 512, 2),
}

# the fused uneven batch (C4): eight processes, sizes 2^U[10, 20] from seed 7 in this order, events
# of process i drawn with seed 7 and stream i
FUSED_SPECS = ["u u~ > g g", "u u~ > g g g", "u u~ > g g g g", "u u~ > g g g g g",
               "u u > u u", "u u > u u g", "u u > u u g g", "u u > u u g g g"]


def fused_sizes(seed: int = 7) -> list:
    rng = np.random.default_rng(seed)
    return [int(2 ** rng.uniform(10, 20)) for _ in FUSED_SPECS]


for _i, (_spec, _n) in enumerate(zip(FUSED_SPECS, fused_sizes())):
    SETS[f"fused_c4_{_i}"] = (_spec, "C2", _n, 7, _i, 64, 3)


def kinematics(name):
    from phasespace import KIN_C1, KIN_C2, KIN_C5
    return {"C1": KIN_C1, "C2": KIN_C2, "C5": KIN_C5}[name]


def sample_indices(n_events: int, n_sample: int, index_seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(index_seed).choice(n_events, n_sample, replace=False))


def momenta_digest(p: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(p, dtype=np.float64).tobytes()).hexdigest()


def _oracle_chunk(task):
    from threadpoolctl import threadpool_limits
    spec, p = task
    with threadpool_limits(limits=1):
        if spec == "g g > g g g g g":
            from oracle.berends_giele import bg_me2
            return bg_me2(spec, p, ALPHA_S)
        from oracle import oracle_me2
        return oracle_me2(spec, p, ALPHA_S)


def write_set(name, pool, workers):
    from phasespace import generate_events
    spec, kin, n, seed, stream, m, iseed = SETS[name]
    nf = len(spec.split(">")[1].split())
    t0 = time.time()
    p = generate_events(n, nf, kinematics(kin), seed=seed, stream=stream)
    idx = sample_indices(n, m, iseed)
    ps = p[idx]
    parts = [ps[w::workers] for w in range(workers)]
    vals = pool.map(_oracle_chunk, [(spec, x) for x in parts])
    me2 = np.empty(m)
    for w in range(workers):
        me2[w::workers] = vals[w]
    path = os.path.join(HERE, f"oracle_{name}.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle |M|^2 of sampled events, written by tests/golden/make_oracle_samples.py "
                "(calls oracle/ and phasespace/ only)\n")
        f.write(f"# spec: {spec}\n# kinematics: {kin}\n# n_events: {n}\n# seed: {seed}\n# stream: {stream}\n")
        f.write(f"# index_seed: {iseed}\n# alpha_s: {ALPHA_S}\n# momenta_sha256: {momenta_digest(ps)}\n")
        for i, v in zip(idx, me2):
            f.write(f"{int(i)} {float(v)!r}\n")
    print(f"[golden] {name}: {m} events of {spec} in {time.time() - t0:.0f}s -> {os.path.basename(path)}",
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*")
    ap.add_argument("--workers", type=int, default=min(8, len(os.sched_getaffinity(0))))
    a = ap.parse_args()
    names = a.only or list(SETS)
    with mp.get_context("fork").Pool(a.workers) as pool:
        for name in names:
            write_set(name, pool, a.workers)


if __name__ == "__main__":
    main()
