"""GPU path vs the oracle over the long horizons of the workloads, in FP64 and in mixed precision.

* The 256-environment superquadric batch (every environment in one batch, as the benchmark runs it):
  eight sampled environments after steps 13 and 26, i.e. through the benchmark's timed window.
* One sampled superquadric environment through its whole 100-step horizon: closing with gravity off,
  gravity on from step 60 (Sec. III-D: gravity is disabled at the start of a grasp), checkpoints 26, 50,
  75, 100.
* The parallel-jaw sphere grasp through all 100 steps: 60 closing, 40 lifting; checkpoints 26, 60, 80,
  100.

The oracle's positions come from tests/golden/oracle_trajectories.npz, written by the committed script
tests/golden/make_oracle_trajectories.py (oracle at PCG tolerance 1e-8; a CPU test checks that the oracle
source has not changed since).  Bars: FP64 (GPU PCG at 1e-8) within 1e-6 of the bbox diagonal; mixed
precision (FP32 PCG storage at tolerance 1e-4, an inexact Newton solve) within 1e-4 through step 26 and
within 1e-3 beyond it: every step stops once |p|_inf <= 1e-5 m/s dt, so two converged solves of a step
differ by a few such increments, and these carry into the following steps through the velocities and, in
contact, through the lagged friction's stick/slip state; over the 100-step grasp that stays under 1e-3 of
the bbox diagonal (the measured values are printed).  A step the oracle fails must fail on the GPU at the
same step with the same reason.
"""
import json
import os

import numpy as np
import pytest

from paper_2503_05020_amd import ipc as G
from paper_2503_05020_amd import scenes as S

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "oracle_trajectories.npz")
META = os.path.join(HERE, "golden", "oracle_trajectories.json")
BAR = {G.IPC_FP64: 1e-6, G.IPC_MIXED: 1e-4}
PCG = {G.IPC_FP64: 1e-8, G.IPC_MIXED: 1e-4}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gold():
    with open(META) as f:
        meta = json.load(f)
    return np.load(GOLD), meta


def _dets(pos, tets):
    x = pos[tets]
    return np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 2))


def _bar(precision, step):
    return BAR[precision] if (precision == G.IPC_FP64 or step <= 26) else 1e-3


def _compare(tag, sc, pos, ref, precision, step, errs):
    err = np.abs(pos - ref).max() / sc["env_bbox_diag"]
    say(f"{tag}: relative position error {err:.2e}")
    errs.append((tag, err, _bar(precision, step)))
    assert _dets(pos, sc["tets"]).min() > 0


def _run(key, scs, gs, steps, gold, precision, checkpoints, which):
    """Steps the batch `gs` one step at a time; at each checkpoint compares the environments in `which`
    (index into gs -> golden case key) with the oracle."""
    data, meta = gold
    fails = {}
    errs = []
    for k in range(1, steps + 1):
        rc, infos = G.ipc_step_batch(gs, 1)
        for j, i in enumerate(infos):
            if i["status"] != 0 and j not in fails:
                fails[j] = (k, i["fail_reason"])
        if k % 10 == 0:
            say(f"{key} step {k}: newton max {max(i['max_newton_iters'] for i in infos)}")
        for j, case in which.items():
            status = data[f"{case}_status"]
            if k <= len(status) and status[k - 1] != 0:
                # the oracle fails this step: the GPU must fail here too, for the same reason
                assert fails.get(j) == (k, int(data[f"{case}_reason"][k - 1])), (case, k, fails.get(j))
                continue
            if k in checkpoints and f"{case}_pos_{k}" in data:
                assert j not in fails, (case, fails[j])
                pos, _ = G.ipc_get_state(gs[j])
                _compare(f"{case} step {k}", scs[j], pos, data[f"{case}_pos_{k}"], precision, k, errs)
    bad = [(t, e, b) for t, e, b in errs if e > b]
    assert not bad, bad


@pytest.mark.parametrize("precision", [G.IPC_FP64, G.IPC_MIXED])
def test_superquadric_batch_through_the_timed_window(precision, gold):
    data, meta = gold
    n_envs = 256
    scs = [S.superquadric_grasp(i) for i in range(n_envs)]
    gs = [G.ipc_create_scene(sc, precision=precision, pcg_rel_tol=PCG[precision]) for sc in scs]
    envs = [int(c.split("_")[1]) for c in meta["cases"] if c.startswith("c3_")]
    assert len(envs) >= 8
    which = {e: f"c3_{e}" for e in envs}
    _run("superquadric batch", scs, gs, 26, gold, precision, {13, 26}, which)
    for g in gs:
        G.ipc_destroy_scene(g)


@pytest.mark.parametrize("precision", [G.IPC_FP64, G.IPC_MIXED])
def test_superquadric_environment_full_horizon(precision, gold):
    data, meta = gold
    full = [c for c, m in meta["cases"].items() if c.startswith("c3_") and 100 in m["checkpoints"]]
    assert len(full) == 1
    e = int(full[0].split("_")[1])
    sc = S.superquadric_grasp(e)
    g = G.ipc_create_scene(sc, precision=precision, pcg_rel_tol=PCG[precision])
    _run("superquadric env", [sc], [g], 100, gold, precision, {26, 50, 75, 100}, {0: full[0]})
    G.ipc_destroy_scene(g)


@pytest.mark.parametrize("precision", [G.IPC_FP64, G.IPC_MIXED])
def test_sphere_grasp_full_horizon(precision, gold):
    sc = S.parallel_jaw_sphere(0)
    g = G.ipc_create_scene(sc, precision=precision, pcg_rel_tol=PCG[precision])
    _run("sphere grasp", [sc], [g], 100, gold, precision, {26, 60, 80, 100}, {0: "c2_0"})
    G.ipc_destroy_scene(g)
