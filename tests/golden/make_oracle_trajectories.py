"""Writes oracle_trajectories.npz: the CPU oracle's positions along long trajectories of the workload
scenes, for the GPU horizon tests (tests/test_gpu_horizons.py).

Only the oracle (oracle/) and the seeded scene generators (paper_2503_05020_amd/scenes.py, which hold no
method arithmetic) are called.  Every trajectory runs the oracle at PCG relative tolerance 1e-8, one step
at a time, and keeps the positions after the listed steps together with each step's status, failure
reason, Newton iterations and active-pair count.  The SHA-256 of the oracle source is stored beside the
data; a CPU test checks that it still matches, so a change of the oracle asks for a rerun of this script:

    python tests/golden/make_oracle_trajectories.py      (about ten minutes on 8 cores)
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_trajectories.npz")
META = os.path.join(HERE, "oracle_trajectories.json")
ORACLE_SRC = os.path.join(ROOT, "oracle", "ipc_oracle.cpp")

# the 256-environment superquadric batch: eight sampled environments through the benchmark's timed window
# (steps 5..24) and beyond, one of them through the whole 100-step horizon (gravity from step 60)
C3_ENVS = [0, 31, 63, 97, 128, 160, 201, 255]
C3_STEPS = 26
C3_FULL_ENV = 128
C3_FULL_CHECKPOINTS = [26, 50, 75, 100]
# the parallel-jaw sphere grasp: closing for 60 steps, lifting for 40
C2_CHECKPOINTS = [26, 60, 80, 100]


def oracle_sha() -> str:
    with open(ORACLE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def jobs():
    out = []
    for e in C3_ENVS:
        cps = C3_FULL_CHECKPOINTS if e == C3_FULL_ENV else [13, C3_STEPS]
        out.append(("c3", e, cps))
    out.append(("c2", 0, C2_CHECKPOINTS))
    return out


def scene(kind, seed):
    from paper_2503_05020_amd import scenes as S
    return S.superquadric_grasp(seed) if kind == "c3" else S.parallel_jaw_sphere(seed)


def run(job):
    import oracle as O
    kind, seed, cps = job
    sc = scene(kind, seed)
    o = O.Scene(sc, pcg_rel_tol=1e-8)
    t0 = time.time()
    rec = {"pos": {}, "status": [], "reason": [], "newton": [], "active": []}
    for k in range(1, max(cps) + 1):
        rc, info = o.step(1)
        rec["status"].append(rc)
        rec["reason"].append(info["fail_reason"])
        rec["newton"].append(info["newton_iters"])
        rec["active"].append(info["n_active_last"])
        if rc != 0:
            break
        if k in cps:
            rec["pos"][k] = o.state()[0]
    print(f"{kind} {seed}: {len(rec['status'])} steps, last rc {rec['status'][-1]}, {time.time() - t0:.0f} s",
          flush=True)
    return job, rec


def main():
    import oracle as O
    O.build()
    js = jobs()
    # longest first
    js.sort(key=lambda j: -max(j[2]))
    with mp.get_context("fork").Pool(min(len(js), os.cpu_count() or 1)) as pool:
        results = pool.map(run, js, chunksize=1)
    arrays, meta = {}, {"oracle_sha256": oracle_sha(), "pcg_rel_tol": 1e-8, "cases": {}}
    for (kind, seed, cps), rec in results:
        key = f"{kind}_{seed}"
        for k, pos in rec["pos"].items():
            arrays[f"{key}_pos_{k}"] = pos
        for f in ("status", "reason", "newton", "active"):
            arrays[f"{key}_{f}"] = np.array(rec[f], np.int64)
        meta["cases"][key] = {"checkpoints": sorted(rec["pos"]), "steps_run": len(rec["status"])}
    np.savez_compressed(OUT, **arrays)
    with open(META, "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
