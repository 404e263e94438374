"""GPU library vs CPU oracle for the solver variants (all off by default) and the per-step contact
statistics:

* the inversion filter (step-size filter keeping every tet inversion-free along the search line,
  Sec. II-C): per-tet cubic det(Ds(x + t p)) and its first root, the scene's step bound, and a press
  trajectory with the filter on;
* repeated friction lagging (the lag count is left open, Sec. III-D);
* adaptive barrier stiffness (Sec. III-D fixes kappa; this is the doubling variant);
* the paper's relative Newton tolerance eps_r (Sec. III-D);
* n_active_last / min_dist_last of every step (the gap behind Table I's D2).

Tolerances: cubic coefficients 1e-12 of their scale, roots and step bounds 1e-9 relative (simple roots:
both sides bisect to adjacent doubles by different rules), positions 1e-6 of the bbox diagonal,
kappa and active-pair counts exactly.
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


def _tets_and_moves(n, seed):
    rng = np.random.default_rng(seed)
    xs, ps = [], []
    while len(xs) < n:
        x = rng.uniform(-1, 1, (4, 3))
        if np.linalg.det((x[1:] - x[0]).T) < 0.2:
            continue
        p = rng.normal(scale=rng.choice([0.1, 0.5, 2.0]), size=(4, 3))
        xs.append(x)
        ps.append(p)
    return np.array(xs), np.array(ps)


def test_tet_first_root_matches_oracle():
    x, p = _tets_and_moves(400, 3)
    tg, kg = G.ipc_debug_tet_first_root(x, p, tmax=1.25)
    finite = 0
    for i in range(len(x)):
        to, ko = O.tet_first_root(x[i], p[i], tmax=1.25)
        scale = np.abs(ko).max()
        assert np.abs(kg[i] - ko).max() <= 1e-12 * scale, i
        if math.isinf(to):
            assert math.isinf(tg[i]), (i, tg[i])
        else:
            finite += 1
            assert tg[i] == pytest.approx(to, rel=1e-9), i
            # the GPU's root is a zero of the cubic (to the rounding of its evaluation)
            assert abs(np.polyval(kg[i][::-1], tg[i])) <= 1e-13 * scale
    say("finite roots", finite, "of", len(x))
    assert finite > 50


def _begin(sc, steps_before, **kw):
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8, **kw)
    o = O.Scene(sc, pcg_rel_tol=1e-8, **kw)
    for _ in range(steps_before):
        assert G.ipc_step(g, 1)[0] == 0
        assert o.step(1)[0] == 0
    xo = o.begin_step()
    G.ipc_debug_begin_step(g)
    return g, o, xo


def test_inversion_bound_matches_oracle():
    """The scene's filter bound along the oracle's Newton direction, and along a direction scaled up until
    it binds."""
    sc = S.press_block(steps=4)
    g, o, xo = _begin(sc, 1)
    po, _ = o.newton_dir(xo)
    bound = 0
    for s in (1.0, 5.0, 25.0, 125.0):
        ag = G.ipc_debug_inversion_bound(g, xo, s * po)
        ao = o.inversion_bound(xo, s * po)
        say(f"scale {s}: gpu {ag:.17g} oracle {ao:.17g}")
        assert ag == pytest.approx(ao, rel=1e-9)
        bound += ao < 1.0
    assert bound >= 1


def test_inversion_filter_trajectory_parity():
    sc = S.press_block(steps=4)
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8, inversion_filter=1)
    o = O.Scene(sc, pcg_rel_tol=1e-8, inversion_filter=1)
    L = sc["env_bbox_diag"]
    tets = sc["tets"]
    for k in range(6):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        assert rg == 0 and ro == 0, (k, ig, io)
        pg, _ = G.ipc_get_state(g)
        po, _ = o.state()
        err = np.abs(pg - po).max() / L
        say(f"step {k}: err {err:.2e} newton {ig['newton_iters']}/{io['newton_iters']}")
        assert err <= 1e-6
        D = np.stack([pg[tets[:, c + 1]] - pg[tets[:, 0]] for c in range(3)], axis=2)
        assert np.linalg.det(D).min() > 0


def test_friction_lagging_parity():
    """A block sliding on a 45 degree incline with three lagged friction updates per step."""
    sc = S.block_on_incline(45.0)
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8, friction_iters=3)
    o = O.Scene(sc, pcg_rel_tol=1e-8, friction_iters=3)
    g1 = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    L = sc["env_bbox_diag"]
    for k in range(10):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        assert G.ipc_step(g1, 1)[0] == 0
        assert rg == 0 and ro == 0, (k, ig, io)
        pg, _ = G.ipc_get_state(g)
        po, _ = o.state()
        err = np.abs(pg - po).max() / L
        say(f"step {k}: err {err:.2e} newton {ig['newton_iters']}/{io['newton_iters']}")
        assert err <= 1e-6
        assert ig["newton_iters"] == io["newton_iters"]
    # the re-lag really changes the trajectory
    p1, _ = G.ipc_get_state(g1)
    assert np.abs(p1 - pg).max() > 1e-9


def test_adaptive_kappa_parity():
    """A light block on a soft barrier (small kappa) sinks below 1e-2 dhat: kappa doubles on both sides at
    the same iterates (same powers of two) and the trajectories agree."""
    sc = S.soft_cube_drop(cells=2, edge=0.02, height=0.0015, kappa=0.005)
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8, adaptive_kappa=1)
    o = O.Scene(sc, pcg_rel_tol=1e-8, adaptive_kappa=1)
    L = sc["env_bbox_diag"]
    k0 = sc["kappa"]
    for k in range(40):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        assert rg == 0 and ro == 0, (k, ig, io)
        assert ig["kappa_last"] == io["kappa_last"], (k, ig["kappa_last"], io["kappa_last"])
        pg, _ = G.ipc_get_state(g)
        po, _ = o.state()
        err = np.abs(pg - po).max() / L
        if k % 8 == 0:
            say(f"step {k}: err {err:.2e} kappa/k0 {ig['kappa_last'] / k0:g}")
        assert err <= 1e-6
    assert ig["kappa_last"] > k0


def test_relative_newton_tolerance_parity():
    """eps_r = 1e-3 of the free-vertex bbox diagonal L (Sec. III-D).  Both sides stop once |p|_inf <= eps_r L dt,
    so a direction a few ulps larger or smaller at that threshold can cost one side one more iteration: per
    step the counts agree within one.  A step that stops one such increment apart leaves positions apart by
    up to eps_r L dt and velocities by eps_r L, which carry into the following steps, so after n steps the
    positions agree within n eps_r dt of the bbox diagonal.  The relative reading never needs more
    iterations than the absolute default."""
    eps_r = 1e-3
    sc = S.soft_cube_drop()
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8, newton_rel_tol=eps_r)
    o = O.Scene(sc, pcg_rel_tol=1e-8, newton_rel_tol=eps_r)
    ga = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    L = sc["env_bbox_diag"]
    n_rel = n_abs = n_or = 0
    worst = 0.0
    for k in range(20):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        ra, ia = G.ipc_step(ga, 1)
        assert rg == 0 and ro == 0 and ra == 0, (k, ig, io)
        assert abs(ig["newton_iters"] - io["newton_iters"]) <= 1, (k, ig, io)
        n_rel += ig["newton_iters"]
        n_or += io["newton_iters"]
        n_abs += ia["newton_iters"]
        pg, _ = G.ipc_get_state(g)
        po, _ = o.state()
        worst = max(worst, np.abs(pg - po).max() / L)
    say(f"newton iterations: relative {n_rel} (oracle {n_or}), absolute {n_abs}; worst position error {worst:.2e}")
    assert worst <= 20 * eps_r * sc["dt"]
    assert n_rel <= n_abs


def test_contact_statistics_match_oracle():
    """Active-pair count (exact) and least active distance (1e-6 relative) after every step of the cube drop."""
    sc = S.soft_cube_drop()
    g = G.ipc_create_scene(sc, pcg_rel_tol=1e-8)
    o = O.Scene(sc, pcg_rel_tol=1e-8)
    seen = 0
    for k in range(20):
        rg, ig = G.ipc_step(g, 1)
        ro, io = o.step(1)
        assert rg == 0 and ro == 0
        assert ig["n_active_last"] == io["n_active_last"], (k, ig, io)
        if io["n_active_last"] == 0:
            assert math.isinf(ig["min_dist_last"]) and math.isinf(io["min_dist_last"])
        else:
            seen += 1
            assert ig["min_dist_last"] == pytest.approx(io["min_dist_last"], rel=1e-6)
            assert 0 < ig["min_dist_last"] < sc["dhat"]
    assert seen > 5


def test_contact_work_counters():
    """ipc_prof_pairs: zero after a reset, no barrier or friction elements without contact, and with
    resting contact at least the last iterate's active pairs per step, classified from more candidates."""
    G.ipc_prof_enable(1)
    try:
        G.ipc_prof_reset()
        assert G.ipc_prof_pairs() == {"candidates": 0, "barrier_elems": 0, "friction_elems": 0}
        g = G.ipc_create_scene(S.free_block())
        assert G.ipc_step(g, 3)[0] == 0
        c = G.ipc_prof_pairs()
        G.ipc_destroy_scene(g)
        assert c["barrier_elems"] == 0 and c["friction_elems"] == 0
        sc = S.soft_cube_drop()
        g = G.ipc_create_scene(sc)
        assert G.ipc_step(g, 14)[0] == 0
        G.ipc_prof_reset()
        rc, info = G.ipc_step(g, 1)
        assert rc == 0 and info["n_active_last"] > 0
        c = G.ipc_prof_pairs()
        G.ipc_destroy_scene(g)
        assert c["barrier_elems"] >= info["n_active_last"]
        assert c["candidates"] >= c["barrier_elems"]
        assert c["friction_elems"] > 0
    finally:
        G.ipc_prof_reset()
        G.ipc_prof_enable(0)
