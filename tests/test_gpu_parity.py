"""GPU library vs CPU oracle, element by element on the same seeded inputs.

Tolerances (see the design notes):
  * candidate and active sets, distance types and squared distances: bit-exact;
  * gradients: |g_gpu - g_oracle|_inf <= 1e-10 * max_i sum_terms |g_term,i| (the
    absolute contributions, because g -> 0 at convergence);
  * Hessian products: 1e-9 of the same scale;
  * positions after a trajectory: max_i |x_gpu - x_oracle| <= 1e-6 * bbox diagonal.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2503_05020_amd import ipc as G
from paper_2503_05020_amd import scenes as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rows(a):
    return {tuple(int(v) for v in r) for r in a}


# ---------------------------------------------------------------------------
# element level
# ---------------------------------------------------------------------------
def _random_pairs(n, seed, kind):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1e-2, 1e-2, (n, 4, 3))
    # a share of near-degenerate configurations: close, parallel, coplanar
    m = n // 4
    x[:m, 0] = x[:m, 1] + rng.normal(scale=1e-6, size=(m, 3))
    x[m:2 * m, 3] = x[m:2 * m, 2] + (x[m:2 * m, 1] - x[m:2 * m, 0]) * 0.5
    x[2 * m:3 * m, :, 2] = 0.0
    return x


@pytest.mark.parametrize("kind", [0, 1])
def test_classify_bit_exact(kind):
    say("classify", kind)
    x = _random_pairs(4000, 11 + kind, kind)
    t, d2 = G.ipc_debug_classify(kind, x.reshape(-1, 12))
    f = O.pt_classify if kind == 0 else O.ee_classify
    for i in range(len(x)):
        to, do = f(x[i])
        assert t[i] == to and d2[i] == do, (i, t[i], to, d2[i], do)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("seed", range(8))
def test_pair_barrier_matches_oracle(kind, seed):
    say("pair barrier", kind, seed)
    rng = np.random.default_rng(300 + seed + 50 * kind)
    dhat, kappa = 1e-3, 3e6
    for _ in range(1000):
        x = rng.uniform(-5e-3, 5e-3, (4, 3))
        x[2:] += rng.normal(size=3) * 1e-3 if kind else 0
        t, d2 = (O.pt_classify if kind == 0 else O.ee_classify)(x)
        if 1e-12 < d2 < dhat * dhat:
            break
        x[0] = (x[1] + x[2] + x[3]) / 3 + rng.normal(size=3) * 3e-4
        t, d2 = (O.pt_classify if kind == 0 else O.ee_classify)(x)
        if 1e-12 < d2 < dhat * dhat:
            break
    eps_x = 1e-3 * np.sum((x[1] - x[0]) ** 2) * np.sum((x[3] - x[2]) ** 2) if kind else 0.0
    if kind and seed % 2:
        eps_x *= 1e6  # force the mollifier branch
    for proj in (False, True):
        eo, go, Ho = O.pair_barrier(kind, t, x, dhat, kappa, eps_x, project=proj)
        eg, gg, Hg = G.ipc_debug_pair_barrier(kind, t, x, dhat, kappa, eps_x, project=proj)
        assert eg == pytest.approx(eo, rel=1e-11, abs=1e-300)
        assert np.abs(gg - go).max() <= 1e-10 * np.abs(go).max() + 1e-300
        assert np.abs(Hg - Ho).max() <= 1e-8 * np.abs(Ho).max() + 1e-300


@pytest.mark.parametrize("seed", range(6))
def test_tet_elastic_matches_oracle(seed):
    say("tet", seed)
    rng = np.random.default_rng(seed)
    X = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0], [0, 0, 0.01]], float)
    x = X + rng.normal(scale=2e-3, size=(4, 3))
    rc, eo, go, Ho = O.tet_elastic(X, x, 1e5, 0.4, project=True)
    if rc != 0:
        pytest.skip("inverted draw")
    rc2, eg, gg, Hg = G.ipc_debug_tet_elastic(X, x, 1e5, 0.4)
    assert rc2 == 0
    assert eg == pytest.approx(eo, rel=1e-11)
    assert np.abs(gg - go).max() <= 1e-10 * np.abs(go).max()
    assert np.abs(Hg - Ho).max() <= 1e-8 * np.abs(Ho).max()


@pytest.mark.parametrize("kind", [0, 1])
def test_accd_matches_oracle(kind):
    say("accd", kind)
    rng = np.random.default_rng(77 + kind)
    x = rng.uniform(-1, 1, (200, 4, 3))
    p = rng.uniform(-2, 2, (200, 4, 3))
    tg = G.ipc_debug_accd(kind, x.reshape(-1, 12), p.reshape(-1, 12))
    to = np.array([O.accd(kind, x[i], p[i]) for i in range(200)])
    assert np.allclose(tg, to, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("kind", [0, 1])
def test_ccd_bound_over_pairs_matches_oracle(kind):
    """min(1, min_k ACCD_k) over pair lists of several sizes (one block, several blocks with a ragged tail,
    empty): equal to the minimum of the oracle's per-pair times (ties broken by the exact minimum)."""
    rng = np.random.default_rng(91 + kind)
    for n in (1, 127, 128, 1000, 4097):
        x = rng.uniform(-1, 1, (n, 4, 3))
        p = rng.uniform(-0.3, 0.3, (n, 4, 3))
        ag = G.ipc_ccd_bound_pairs(kind, x.reshape(-1, 12), p.reshape(-1, 12))
        ao = min(1.0, min(O.accd(kind, x[i], p[i]) for i in range(n)))
        say(f"kind {kind} n {n}: gpu {ag:.17g} oracle {ao:.17g}")
        assert ag == pytest.approx(ao, rel=1e-9, abs=1e-15)
        # the pair holding the minimum gives the same time alone
        if ao < 1.0:
            i = int(np.argmin([O.accd(kind, x[j], p[j]) for j in range(n)]))
            assert G.ipc_ccd_bound_pairs(kind, x[i:i + 1].reshape(-1, 12), p[i:i + 1].reshape(-1, 12)) == ag
    assert G.ipc_ccd_bound_pairs(kind, np.zeros((0, 12)), np.zeros((0, 12))) == 1.0


# ---------------------------------------------------------------------------
# scene level
# ---------------------------------------------------------------------------
def _pair_scenes():
    return {
        "two_tets": S.two_tets(gap=0.0006),
        "cube_small": S.soft_cube_drop(cells=3, edge=0.06, height=0.0004),
    }


@pytest.mark.parametrize("name", ["two_tets", "cube_small"])
def test_candidates_and_active_sets_bit_exact(name):
    say("sets", name)
    sc = _pair_scenes()[name]
    g = G.ipc_create_scene(sc)
    o = O.Scene(sc)
    rng = np.random.default_rng(5)
    x = sc["rest_pos"] + rng.normal(scale=1e-4, size=sc["rest_pos"].shape) * (sc["kin_group"] < 0)[:, None]
    assert rows(G.ipc_debug_candidates(g, x)) == rows(O.Scene.candidates(o, x))
    p = rng.normal(scale=1e-3, size=x.shape) * (sc["kin_group"] < 0)[:, None]
    assert rows(G.ipc_debug_candidates(g, x, p)) == rows(o.candidates(x, p))
    ag, dg = G.ipc_debug_active(g, x)
    ao, do = o.active(x)
    assert len(ag) > 0
    mg = {tuple(r[:5]): (r[5], d) for r, d in zip(ag.tolist(), dg)}
    mo = {tuple(r[:5]): (r[5], d) for r, d in zip(ao.tolist(), do)}
    assert mg == mo


@pytest.mark.parametrize("name", ["sphere", "superquadric7"])
def test_candidate_sets_bit_exact_on_workload_scenes(name):
    """Grid broad phase vs the oracle's all-pairs test on scenes with huge (ground) and rotated primitives."""
    say("workload sets", name)
    sc = S.parallel_jaw_sphere() if name == "sphere" else S.superquadric_grasp(7)
    g = G.ipc_create_scene(sc)
    o = O.Scene(sc)
    rng = np.random.default_rng(9)
    free = (sc["kin_group"] < 0)[:, None]
    # squeeze the scene a little so that many pairs come within dhat
    c = sc["rest_pos"][free[:, 0]].mean(0)
    x = sc["rest_pos"] + (c - sc["rest_pos"]) * 0.01 * free + rng.normal(scale=2e-4, size=sc["rest_pos"].shape) * free
    assert rows(G.ipc_debug_candidates(g, x)) == rows(o.candidates(x))
    p = rng.normal(scale=2e-3, size=x.shape) * free
    assert rows(G.ipc_debug_candidates(g, x, p)) == rows(o.candidates(x, p))
    big = rng.normal(scale=3e-2, size=x.shape) * free  # large sweeps take the all-pairs path
    assert rows(G.ipc_debug_candidates(g, x, big)) == rows(o.candidates(x, big))
    ag, dg = G.ipc_debug_active(g, x)
    ao, do = o.active(x)
    assert {tuple(r) for r in ag.tolist()} == {tuple(r) for r in ao.tolist()}
    assert sorted(dg.tolist()) == sorted(do.tolist())


def _begin(sc, steps_before=0, **kw):
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8, **kw)
    o = O.Scene(sc, pcg_rel_tol=1e-8, **kw)
    for _ in range(steps_before):
        assert G.ipc_step(g, 1)[0] == 0
        assert o.step(1)[0] == 0
    pg, vg = G.ipc_get_state(g)
    o.set_state(pg, vg, o.step_index)  # identical state on both sides
    xg = G.ipc_debug_begin_step(g)
    xo = o.begin_step()
    return g, o, xg, xo


@pytest.mark.parametrize("steps_before", [0, 6])
def test_gradient_hessian_energy_parity(steps_before):
    say("gradient parity", steps_before)
    sc = S.soft_cube_drop(cells=3, edge=0.06, height=0.002)
    g, o, xg, xo = _begin(sc, steps_before)
    assert np.array_equal(xg, xo)
    free = (sc["kin_group"] < 0)[:, None]
    rng = np.random.default_rng(steps_before)
    for k in range(3):
        x = xo + rng.normal(scale=2e-5, size=xo.shape) * free * (k > 0)
        gg = G.ipc_debug_gradient(g, x)
        go, gabs = o.gradient(x)
        scale = gabs.max()
        assert np.abs(gg - go).max() <= 1e-10 * scale, (np.abs(gg - go).max(), scale)
        v = rng.normal(size=x.shape) * free
        yg = G.ipc_debug_hessian_apply(g, x, v)
        H = o.hessian_dense(x)
        yo = (H @ v.reshape(-1)).reshape(-1, 3)
        assert np.abs(yg - yo).max() <= 1e-9 * np.abs(yo).max()
        eg, eo = G.ipc_debug_energy(g, x), o.energy(x)
        assert eg == pytest.approx(eo, rel=1e-12)


def test_newton_direction_and_ccd_parity():
    say("newton dir")
    sc = S.soft_cube_drop(cells=3, edge=0.06, height=0.002)
    g, o, xg, xo = _begin(sc, 3)
    pg, itg = G.ipc_debug_newton_dir(g, xo)
    po, ito = o.newton_dir(xo)
    assert np.abs(pg - po).max() <= 1e-6 * np.abs(po).max()
    ag = G.ipc_debug_ccd_bound(g, xo, po)
    ao = o.ccd_bound(xo, po)
    assert ag == pytest.approx(ao, rel=1e-9)


def test_cube_drop_trajectory_parity():
    """Soft cube drop: 50 steps, positions within 1e-6 of the bbox diagonal (Table I: no penetration)."""
    sc = S.soft_cube_drop()
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    o = O.Scene(sc, pcg_rel_tol=1e-8)
    L = sc["env_bbox_diag"]
    worst = 0.0
    for k in range(50):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        assert rg == 0 and ro == 0, (k, ig, io)
        pg, vg = G.ipc_get_state(g)
        po, vo = o.state()
        err = np.abs(pg - po).max() / L
        worst = max(worst, err)
        if k % 10 == 0:
            say(f"step {k}: err {err:.2e} newton {ig['newton_iters']}/{io['newton_iters']} pcg {ig['pcg_iters']}")
    say("worst", worst)
    assert worst <= 1e-6
    # zero penetration: the last configuration is valid
    assert pg[: len(pg) - 4, 2].min() > 0


def test_augmented_lagrangian_press_parity():
    """Plate pressed onto a block faster than the gap allows: the augmented-Lagrangian Dirichlet mode
    (the reading taken for enforcing prescribed finger motion, Sec. III-D; the paper names no method) must end each step with the plate on target and match the oracle's trajectory."""
    sc = S.press_block(steps=4)
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    o = O.Scene(sc, pcg_rel_tol=1e-8)
    kin = sc["kin_group"]
    X = sc["rest_pos"]
    L = sc["env_bbox_diag"]
    for k in range(6):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        assert rg == 0 and ro == 0, (k, ig, io)
        pg, _ = G.ipc_get_state(g)
        po, _ = o.state()
        err = np.abs(pg - po).max() / L
        say(f"step {k}: err {err:.2e} newton {ig['newton_iters']}/{io['newton_iters']}")
        assert err <= 1e-6
        target = X[kin == 1, 2] - 0.3 * sc["dt"] * min(k + 1, 4)
        assert np.array_equal(pg[kin == 1, 2], target)
        assert pg[kin < 0, 2].max() < target.min()
    x = pg[sc["tets"]]
    assert np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 2)).min() > 0


@pytest.mark.parametrize("precision", [G.IPC_FP64, G.IPC_MIXED])
def test_pcg_paths_same_bits(precision):
    """Tiled PCG, tiled with the per-environment tail hand-off at the first poll, and the fully
    per-environment PCG reduce in the same order: the trajectories must be bitwise identical."""
    scs = [S.soft_cube_drop(cells=3, edge=0.05, height=0.003 + 0.001 * i, seed=i) for i in range(3)]
    runs = []
    # the per-environment kernels are block Jacobi only: compare with the two-level PCG off
    G.ipc_set_tuning(G.IPC_TUNE_COARSE, 0)
    for tail, fused in ((0, 0), (1 << 30, 0), (0, 1)):
        G.ipc_set_tuning(G.IPC_TUNE_TAIL_TILES, tail)
        G.ipc_set_tuning(G.IPC_TUNE_FUSED_PCG, fused)
        gs = [G.ipc_create_scene(sc, precision=precision) for sc in scs]
        for _ in range(8):
            rc, _ = G.ipc_step_batch(gs, 1)
            assert rc == 0
        runs.append([G.ipc_get_state(g)[0] for g in gs])
        for g in gs:
            G.ipc_destroy_scene(g)
    G.ipc_set_tuning(G.IPC_TUNE_TAIL_TILES, 0)
    G.ipc_set_tuning(G.IPC_TUNE_FUSED_PCG, 0)
    G.ipc_set_tuning(G.IPC_TUNE_COARSE, 1)
    for k in (1, 2):
        for a, b in zip(runs[0], runs[k]):
            assert np.array_equal(a, b), k


def test_lane_count_changes_no_result():
    """The same batch placed on one lane and spread over four lanes (one stream and one host
    thread each) gives bitwise identical trajectories: every reduction is environment-local."""
    scs = [S.soft_cube_drop(cells=2, edge=0.04, height=0.002 + 0.001 * i, seed=i) for i in range(6)]
    before = G.ipc_get_tuning(G.IPC_TUNE_LANES)
    runs = []
    try:
        for lanes in (1, 4):
            G.ipc_set_tuning(G.IPC_TUNE_LANES, lanes)
            gs = [G.ipc_create_scene(sc) for sc in scs]
            rc, infos = G.ipc_step_batch(gs, 5)
            assert rc == 0, infos
            runs.append([G.ipc_get_state(g)[0] for g in gs])
            for g in gs:
                G.ipc_destroy_scene(g)
    finally:
        G.ipc_set_tuning(G.IPC_TUNE_LANES, before)
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)


def _async_batch(precision):
    """Environments whose steps take different Newton iteration counts: cube drops at different heights
    (impact at different steps), a plate pressed faster than the gap allows (augmented-Lagrangian
    Dirichlet mode), a block sliding on an incline with two lagged friction updates per step, a cube
    with the inversion filter and adaptive kappa, and one that fails (one Newton iteration allowed)."""
    scs = [S.soft_cube_drop(cells=2, edge=0.04, height=0.002 + 0.002 * i, seed=i) for i in range(4)]
    scs.append(S.press_block(steps=4))
    inc = S.block_on_incline(45.0)
    inc["friction_iters"] = 2
    scs.append(inc)
    var = S.soft_cube_drop(cells=2, edge=0.02, height=0.0015, kappa=0.005, seed=7)
    var["inversion_filter"] = 1
    var["adaptive_kappa"] = 1
    scs.append(var)
    bad = S.soft_cube_drop(cells=2, edge=0.04, height=0.001, seed=9)
    bad["newton_max_iter"] = 1
    scs.append(bad)
    return scs


@pytest.mark.parametrize("precision", [G.IPC_FP64, G.IPC_MIXED])
def test_decoupled_schedule_same_bits_as_lock_step(precision):
    """Within a lane, environments that finish a step begin the next while the others still iterate
    (IPC_TUNE_ASYNC = 1): every environment runs the same sequence as under lock-step time steps, so
    positions, velocities and per-step records are bitwise equal, failure included."""
    scs = _async_batch(precision)
    before = G.ipc_get_tuning(G.IPC_TUNE_ASYNC)
    runs = []
    try:
        for mode in (0, 1):
            G.ipc_set_tuning(G.IPC_TUNE_ASYNC, mode)
            gs = [G.ipc_create_scene(sc, precision=precision, pcg_rel_tol=1e-6) for sc in scs]
            recs = []
            for chunk in (3, 5):  # two calls: the second starts from the state the first left
                rc, infos = G.ipc_step_batch(gs, chunk)
                recs.append(infos)
            say(f"mode {mode}:", [i["steps_done"] for i in recs[0]], [i["newton_iters"] for i in recs[1]])
            runs.append(([G.ipc_get_state(g) for g in gs], recs))
            for g in gs:
                G.ipc_destroy_scene(g)
    finally:
        G.ipc_set_tuning(G.IPC_TUNE_ASYNC, before)
    (st0, rec0), (st1, rec1) = runs
    assert rec0[0][-1]["status"] != 0 and rec0[0][-1]["fail_reason"] == 1  # the failing one
    for (p0, v0), (p1, v1) in zip(st0, st1):
        assert np.array_equal(p0, p1) and np.array_equal(v0, v1)
    for a, b in zip(rec0, rec1):
        for i0, i1 in zip(a, b):
            for k in ("steps_done", "status", "fail_reason", "newton_iters", "max_newton_iters", "ls_halvings",
                      "pcg_iters", "n_active_last", "kappa_last"):
                assert i0[k] == i1[k], (k, i0, i1)
            assert i0["min_dist_last"] == i1["min_dist_last"] or (np.isinf(i0["min_dist_last"])
                                                                  and np.isinf(i1["min_dist_last"]))


def test_decoupled_schedule_superquadric_batch_same_bits():
    """The benchmark's workload (first 32 environments, mixed precision) over 8 steps through first contact:
    decoupled and lock-step schedules give the same bits."""
    scs = [S.superquadric_grasp(i) for i in range(32)]
    before = G.ipc_get_tuning(G.IPC_TUNE_ASYNC)
    runs = []
    try:
        for mode in (0, 1):
            G.ipc_set_tuning(G.IPC_TUNE_ASYNC, mode)
            gs = [G.ipc_create_scene(sc, precision=G.IPC_MIXED, pcg_rel_tol=1e-4) for sc in scs]
            G.ipc_step_batch(gs, 6)
            rc, infos = G.ipc_step_batch(gs, 8)
            runs.append(([G.ipc_get_state(g)[0] for g in gs], [i["newton_iters"] for i in infos]))
            for g in gs:
                G.ipc_destroy_scene(g)
    finally:
        G.ipc_set_tuning(G.IPC_TUNE_ASYNC, before)
    assert runs[0][1] == runs[1][1]
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)


def test_alone_equals_batch_bitwise():
    say("alone vs batch")
    scs = [S.soft_cube_drop(cells=2, edge=0.04, height=0.002 + 0.001 * i, seed=i) for i in range(3)]
    alone = []
    for sc in scs:
        g = G.ipc_create_scene(sc)
        assert G.ipc_step(g, 4)[0] == 0
        alone.append(G.ipc_get_state(g)[0])
    gs = [G.ipc_create_scene(sc) for sc in scs]
    rc, infos = G.ipc_step_batch(gs, 4)
    assert rc == 0, infos
    for a, g in zip(alone, gs):
        assert np.array_equal(a, G.ipc_get_state(g)[0])


def test_failure_is_isolated():
    say("failure isolation")
    scs = [S.soft_cube_drop(cells=2, edge=0.04, height=0.002, seed=i) for i in range(3)]
    solo = G.ipc_create_scene(scs[2])
    G.ipc_step(solo, 3)
    ref = G.ipc_get_state(solo)[0]
    gs = [G.ipc_create_scene(scs[0]), G.ipc_create_scene(scs[1], newton_max_iter=1), G.ipc_create_scene(scs[2])]
    before = G.ipc_get_state(gs[1])[0]
    rc, infos = G.ipc_step_batch(gs, 3)
    assert rc == G.IPC_E_FAILED
    assert infos[1]["status"] == G.IPC_E_FAILED and infos[1]["fail_reason"] == 1
    assert infos[0]["status"] == 0 and infos[2]["status"] == 0
    assert np.array_equal(G.ipc_get_state(gs[2])[0], ref)
    assert np.array_equal(G.ipc_get_state(gs[1])[0], before)  # frozen at its last accepted step
    rc, _ = G.ipc_step(gs[1], 1)
    assert rc == G.IPC_E_FAILED


def test_create_rejects_bad_scenes():
    say("bad scenes")
    sc = S.soft_cube_drop(cells=2, edge=0.04)
    bad = dict(sc)
    bad["tets"] = sc["tets"][:, [1, 0, 2, 3]].copy()
    with pytest.raises(G.IPCError) as e:
        G.ipc_create_scene(bad)
    assert e.value.code == G.IPC_E_INVERTED
    bad = dict(sc)
    bad["init_pos"] = sc["rest_pos"].copy()
    bad["init_pos"][:-4, 2] -= 0.03
    with pytest.raises(G.IPCError) as e:
        G.ipc_create_scene(bad)
    assert e.value.code == G.IPC_E_INTERSECTING
    bad = dict(sc)
    bad["dhat"] = -1.0
    with pytest.raises(G.IPCError) as e:
        G.ipc_create_scene(bad)
    assert e.value.code == G.IPC_E_ARG


def test_stress_output_matches_oracle():
    say("stress")
    sc = S.soft_cube_drop(cells=3, edge=0.06, height=0.0015)
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    o = O.Scene(sc, pcg_rel_tol=1e-8)
    for _ in range(8):
        G.ipc_step(g, 1)
        o.step(1)
    pg, vg, cg, mg = G.ipc_get_state(g, stress=True)
    o.set_state(pg, vg, o.step_index)
    po, vo, co, mo = o.state(stress=True)
    assert np.allclose(cg, co, rtol=1e-10, atol=1e-10 * np.abs(co).max())
    assert np.allclose(mg, mo, rtol=1e-10, atol=1e-10 * np.abs(mo).max())
