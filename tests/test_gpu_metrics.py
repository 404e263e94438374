"""Grasp-quality metrics D1 / D2 (Sec. IV-C, Eq. (2)-(3)) on the GPU against the oracle
(oracle/metrics.py):

* cube on the ground, ground triangles as the 'gripper': every sample's signed distance within 1e-12
  of the oracle's (absolute, metres) and D1 / D2 equal;
* the same cube pushed through the ground by a known depth with ipc_set_state: D1 = D2 = that depth
  (the penetration branch of Fig. 6);
* the parallel-jaw sphere grasp in contact, 50,000 samples on the two fingers (the paper's count): a
  seeded subset of samples against the oracle one by one, D1 = 0 (no penetration, Table I) and
  0 < D2 < dhat (a tight grasp, Table I's D2 ~ dhat).
"""
import numpy as np
import pytest

import oracle as O
from oracle import metrics as M
from paper_2503_05020_amd import ipc as G
from paper_2503_05020_amd import scenes as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_metrics_cube_on_ground_match_oracle():
    sc = S.soft_cube_drop(cells=3, edge=0.06, height=0.0015)
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    for _ in range(10):
        assert G.ipc_step(g, 1)[0] == 0
    pos, _ = G.ipc_get_state(g)
    obj = S.body_surface(sc, 0)
    ground = S.body_surface(sc, 1)
    st, uv = S.surface_samples(sc, ground, 2000, seed=4)
    D1, D2, sdf = G.ipc_grasp_metrics(g, obj, ground, st, uv, want_sdf=True)
    o1, o2, od = M.grasp_metrics(pos, obj, ground, st, uv)
    say(f"gpu D1 {D1:.3e} D2 {D2:.6e}; oracle D1 {o1:.3e} D2 {o2:.6e}")
    assert np.abs(sdf - od).max() <= 1e-12
    assert D1 == o1 == 0.0
    assert D2 == pytest.approx(o2, abs=1e-15)
    assert 0 < D2 < 0.5  # the nearest ground sample is outside the cube


def test_metrics_penetration_depth():
    sc = S.soft_cube_drop(cells=3, edge=0.06, height=0.0015)
    g = G.ipc_create_scene(sc)
    pos = sc["rest_pos"].copy()
    obj = S.body_surface(sc, 0)
    ground = S.body_surface(sc, 1)
    zmin = pos[sc["kin_group"] < 0, 2].min()
    # samples on a small square of the ground right under the cube's bottom face
    st, uv = S.surface_samples(sc, ground, 4000, seed=5)
    for depth in (0.004, 0.0011):
        p = pos.copy()
        p[sc["kin_group"] >= 0, 2] = zmin + depth  # the ground plane lifted into the cube
        G.ipc_set_state(g, p)
        D1, D2, sdf = G.ipc_grasp_metrics(g, obj, ground, st, uv, want_sdf=True)
        o1, o2, od = M.grasp_metrics(p, obj, ground, st, uv)
        say(f"depth {depth}: gpu D1 {D1:.6e} D2 {D2:.6e}; oracle {o1:.6e} {o2:.6e}")
        assert np.abs(sdf - od).max() <= 1e-12
        assert D1 == pytest.approx(o1, abs=1e-15) and D2 == pytest.approx(o2, abs=1e-15)
        # the deepest ground sample under the cube is `depth` inside it (cube bottom face is flat: the jitter
        # moves it by at most 1e-4)
        assert D1 == D2
        assert D1 == pytest.approx(depth, abs=2e-4)


def test_metrics_sphere_grasp_50k_samples():
    sc = S.parallel_jaw_sphere()
    g = G.ipc_create_scene(sc, precision=G.IPC_MIXED)
    rc, info = G.ipc_step(g, 26)
    assert rc == 0 and info["n_active_last"] > 0
    pos, _ = G.ipc_get_state(g)
    obj = S.body_surface(sc, 0)
    fingers = np.concatenate([S.body_surface(sc, 1), S.body_surface(sc, 2)])
    st, uv = S.surface_samples(sc, fingers, 50000, seed=6)
    D1, D2, sdf = G.ipc_grasp_metrics(g, obj, fingers, st, uv, want_sdf=True)
    rng = np.random.default_rng(7)
    pick = rng.choice(len(st), 300, replace=False)
    pick = np.concatenate([pick, [int(np.argmax(sdf))]])  # and the sample that decides D1 / D2
    od = M.signed_distance(M.sample_points(pos, fingers, st[pick], uv[pick]), pos, obj)
    say(f"sphere grasp: D1 {D1:.3e} D2 {D2 * 100:.4f} cm (dhat {sc['dhat'] * 100} cm), "
        f"sampled |sdf - oracle| {np.abs(sdf[pick] - od).max():.2e}")
    assert np.abs(sdf[pick] - od).max() <= 1e-12
    assert D1 == 0.0
    assert 0.0 < D2 < sc["dhat"]
    assert D2 == pytest.approx(abs(sdf.max()), abs=0)
