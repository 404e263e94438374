"""Pins of the CPU oracle against what mathematics and the paper fix.

None of these tests compares the oracle with itself: each checks a closed
form, a finite difference, a brute-force search, a library routine (numpy's
symmetric eigensolver), an exact physical solution or a value the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2503_05020_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1234)


# ---------------------------------------------------------------------------
# paper constants (Sec. III-D) and defaults of the workloads
# ---------------------------------------------------------------------------
def test_defaults_match_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    p = S.DEFAULT_PARAMS
    assert p["dt"] == g["dt"] and p["kappa"] == g["kappa"] and p["dhat"] == g["dhat"]
    assert p["eps_v"] == g["eps_v"] and p["newton_max_iter"] == g["newton_max_iter"]


# ---------------------------------------------------------------------------
# barrier b(d) = -(d - dhat)^2 ln(d/dhat)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [1e-6, 1e-5, 3e-4, 7e-4, 9.99e-4])
def test_barrier_closed_form_and_fd(d):
    dhat = 1e-3
    b = O.barrier_scalar(d, dhat)
    assert b[0] == pytest.approx(-(d - dhat) ** 2 * math.log(d / dhat), rel=1e-14)
    h = d * 1e-5
    fd1 = (O.barrier_scalar(d + h, dhat)[0] - O.barrier_scalar(d - h, dhat)[0]) / (2 * h)
    fd2 = (O.barrier_scalar(d + h, dhat)[1] - O.barrier_scalar(d - h, dhat)[1]) / (2 * h)
    assert b[1] == pytest.approx(fd1, rel=1e-6)
    assert b[2] == pytest.approx(fd2, rel=1e-6)
    assert b[0] > 0 and b[1] < 0 and b[2] > 0


def test_barrier_c2_at_dhat():
    dhat = 1e-3
    assert np.all(O.barrier_scalar(dhat, dhat) == 0)
    left = O.barrier_scalar(dhat * (1 - 1e-7), dhat)
    assert abs(left[0]) < 1e-20 and abs(left[1]) < 1e-13 and abs(left[2]) < 1e-6
    assert np.all(O.barrier_scalar(2 * dhat, dhat) == 0)


# ---------------------------------------------------------------------------
# friction smoothing f0
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("y", [0.0, 1e-7, 3e-6, 9e-6, 1e-5, 2e-5, 1e-3])
def test_friction_f0(y):
    eps = 1e-5
    f = O.friction_f0(y, eps)
    if y < eps:
        assert f[0] == pytest.approx(-y ** 3 / (3 * eps ** 2) + y * y / eps + eps / 3, rel=1e-14)
    else:
        assert f[0] == y and f[1] == 1 and f[2] == 0
    if y > 1e-7:
        h = 1e-9
        fd = (O.friction_f0(y + h, eps)[0] - O.friction_f0(y - h, eps)[0]) / (2 * h)
        assert f[1] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_friction_f0_continuity_at_eps():
    eps = 1e-5
    a, b = O.friction_f0(eps * (1 - 1e-12), eps), O.friction_f0(eps, eps)
    assert a[0] == pytest.approx(b[0], rel=1e-10)
    assert a[1] == pytest.approx(b[1], rel=1e-10)
    assert abs(a[2]) < 1e-5  # f1' -> 0 at eps (C1 friction force)
    assert O.friction_f0(0.0, eps)[1] == 0.0


# ---------------------------------------------------------------------------
# distances: brute force over dense parameter grids
# ---------------------------------------------------------------------------
def _pt_sampled(x, n=300):
    p, t0, t1, t2 = x
    u = np.linspace(0, 1, n)
    B1, B2 = np.meshgrid(u, u, indexing="ij")
    m = B1 + B2 <= 1
    q = t0 + B1[m, None] * (t1 - t0) + B2[m, None] * (t2 - t0)
    return ((q - p) ** 2).sum(1).min()


def _ee_sampled(x, n=300):
    a0, a1, b0, b1 = x
    u = np.linspace(0, 1, n)
    A = a0 + u[:, None] * (a1 - a0)
    B = b0 + u[:, None] * (b1 - b0)
    return ((A[:, None, :] - B[None, :, :]) ** 2).sum(2).min()


@pytest.mark.parametrize("seed", range(40))
def test_pt_distance_vs_sampling(seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (4, 3))
    if seed % 4 == 0:  # point just above the triangle interior
        x[0] = (x[1] + x[2] + x[3]) / 3 + 1e-3 * np.cross(x[2] - x[1], x[3] - x[1])
    t, d2 = O.pt_classify(x)
    sm = _pt_sampled(x)
    emax = max(np.linalg.norm(x[i] - x[j]) for i in range(1, 4) for j in range(1, 4))
    assert d2 <= sm * (1 + 1e-12) + 1e-15
    assert math.sqrt(sm) - math.sqrt(d2) <= 2.5 * emax / 300
    assert 0 <= t <= 6


@pytest.mark.parametrize("seed", range(40))
def test_ee_distance_vs_sampling(seed):
    rng = np.random.default_rng(100 + seed)
    x = rng.uniform(-1, 1, (4, 3))
    if seed % 5 == 0:  # nearly parallel edges
        x[3] = x[2] + (x[1] - x[0]) * 0.7 + 1e-5
    t, d2 = O.ee_classify(x)
    sm = _ee_sampled(x)
    emax = max(np.linalg.norm(x[1] - x[0]), np.linalg.norm(x[3] - x[2]))
    assert d2 <= sm * (1 + 1e-12) + 1e-15
    assert math.sqrt(sm) - math.sqrt(d2) <= 2.5 * emax / 300
    assert 0 <= t <= 8


def test_distance_type_special_cases():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    t, d2 = O.pt_classify(np.vstack([[0.2, 0.2, 0.5], tri]))
    assert t == 0 and d2 == pytest.approx(0.25)
    t, d2 = O.pt_classify(np.vstack([[0.5, -1.0, 0.0], tri]))
    assert t == 1 and d2 == pytest.approx(1.0)  # edge (t0,t1)
    t, d2 = O.pt_classify(np.vstack([[-1.0, -1.0, 0.0], tri]))
    assert t == 4 and d2 == pytest.approx(2.0)  # vertex t0
    t, d2 = O.ee_classify(np.array([[0, 0, 0], [1, 0, 0], [0.5, -1, 1], [0.5, 1, 1]], float))
    assert t == 0 and d2 == pytest.approx(1.0)
    t, d2 = O.ee_classify(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float))
    assert t != 0 and d2 == pytest.approx(1.0)  # parallel edges fall back


# ---------------------------------------------------------------------------
# pair barrier: AD derivatives against central differences
# ---------------------------------------------------------------------------
def _fd_grad(f, x, h):
    g = np.zeros(x.size)
    for i in range(x.size):
        e = np.zeros(x.size)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def _near_pair(kind, rng, dhat):
    for _ in range(1000):
        x = rng.uniform(-0.01, 0.01, (4, 3))
        if kind == 0:
            c = (x[1] + x[2] + x[3]) / 3
            n = np.cross(x[2] - x[1], x[3] - x[1])
            x[0] = c + n / np.linalg.norm(n) * rng.uniform(0.2, 0.9) * dhat + rng.normal(size=3) * 1e-3
            t, d2 = O.pt_classify(x)
        else:
            n = np.cross(x[1] - x[0], x[3] - x[2])
            mid_a, mid_b = (x[0] + x[1]) / 2, (x[2] + x[3]) / 2
            shift = mid_a - mid_b + n / np.linalg.norm(n) * rng.uniform(0.2, 0.9) * dhat
            x[2:] += shift
            t, d2 = O.ee_classify(x)
        if 0 < d2 < dhat * dhat:
            return x, t
    raise RuntimeError("no pair")


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("seed", range(6))
def test_pair_barrier_derivatives_fd(kind, seed):
    rng = np.random.default_rng(seed + 10 * kind)
    dhat, kappa = 1e-3, 3e6
    x, t = _near_pair(kind, rng, dhat)
    # big threshold so the EE mollifier is active for some seeds
    eps_x = 0.0 if kind == 0 else (1e-9 if seed % 2 else 1e-14)
    e, g, H = O.pair_barrier(kind, t, x, dhat, kappa, eps_x)
    assert e > 0
    x0 = x.reshape(-1)

    def en(y):
        return O.pair_barrier(kind, t, y.reshape(4, 3), dhat, kappa, eps_x)[0]

    def gr(y):
        return O.pair_barrier(kind, t, y.reshape(4, 3), dhat, kappa, eps_x)[1]

    h = 1e-9
    fg = _fd_grad(en, x0, h)
    assert np.allclose(g, fg, rtol=1e-5, atol=1e-6 * np.abs(g).max())
    fH = np.stack([_fd_grad(lambda y, i=i: gr(y)[i], x0, h) for i in range(12)])
    assert np.allclose(H, fH, rtol=1e-4, atol=1e-5 * np.abs(H).max())
    assert np.allclose(H, H.T, atol=1e-9 * np.abs(H).max())


def test_mollifier_edge_parallel_energy_vanishes():
    # exactly parallel edges: c = 0 -> mollifier 0 -> zero energy
    x = np.array([[0, 0, 0], [1e-2, 0, 0], [2e-3, 5e-4, 0], [8e-3, 5e-4, 0]], float)
    t, d2 = O.ee_classify(x)
    e, g, H = O.pair_barrier(1, t, x, 1e-3, 3e6, 1e-3 * 1e-4 * 3.6e-5)
    assert e == 0.0


# ---------------------------------------------------------------------------
# Neo-Hookean: textbook cases
# ---------------------------------------------------------------------------
X_REF = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0], [0, 0, 0.01]], float)


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_neohookean_rest_state():
    E, nu = 1e5, 0.4
    rc, e, g, H = O.tet_elastic(X_REF, X_REF, E, nu)
    assert rc == 0 and abs(e) < 1e-18 and np.abs(g).max() < 1e-14
    mu, la = E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))
    # linear elasticity: H = V B^T C B with C_ijkl = mu (d_ik d_jl + d_il d_jk) + la d_ij d_kl
    C = np.zeros((9, 9))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    C[3 * i + j, 3 * k + l] = mu * ((i == k) * (j == l) + (i == l) * (j == k)) + la * (i == j) * (k == l)
    Dm = (X_REF[1:] - X_REF[0]).T
    Dinv = np.linalg.inv(Dm)
    B = np.zeros((9, 12))
    for i in range(3):
        for j in range(3):
            for a in range(3):
                B[3 * i + j, 3 * (a + 1) + i] = Dinv[a, j]
            B[3 * i + j, i] = -Dinv[:, j].sum()
    V = np.linalg.det(Dm) / 6
    assert np.allclose(H, V * B.T @ C @ B, rtol=1e-10, atol=1e-12 * np.abs(H).max())


@pytest.mark.parametrize("s", [0.7, 0.95, 1.3, 2.0])
def test_neohookean_uniaxial(s):
    E, nu = 2e5, 0.3
    mu, la = E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))
    x = X_REF.copy()
    x[:, 0] *= s
    rc, e, g, H = O.tet_elastic(X_REF, x, E, nu)
    V = 1e-6 / 6
    assert e == pytest.approx(V * (mu / 2 * (s * s - 1) - mu * math.log(s) + la / 2 * math.log(s) ** 2), rel=1e-12)


def test_neohookean_rotation_invariance_and_fd():
    rng = np.random.default_rng(7)
    E, nu = 1e5, 0.45
    x = X_REF + rng.normal(scale=1e-3, size=(4, 3))
    R = _rot(rng)
    rc, e, g, H = O.tet_elastic(X_REF, x, E, nu)
    rc2, e2, g2, _ = O.tet_elastic(X_REF, x @ R.T + 0.3, E, nu)
    assert e2 == pytest.approx(e, rel=1e-12)
    assert np.allclose(g2.reshape(4, 3), g.reshape(4, 3) @ R.T, atol=1e-10 * np.abs(g).max())
    x0 = x.reshape(-1)
    fg = _fd_grad(lambda y: O.tet_elastic(X_REF, y.reshape(4, 3), E, nu)[1], x0, 1e-8)
    assert np.allclose(g, fg, rtol=1e-5, atol=1e-6 * np.abs(g).max())
    fH = np.stack([_fd_grad(lambda y, i=i: O.tet_elastic(X_REF, y.reshape(4, 3), E, nu)[2][i], x0, 1e-8)
                   for i in range(12)])
    assert np.allclose(H, fH, rtol=1e-4, atol=1e-5 * np.abs(H).max())


def test_inverted_tet_is_infeasible():
    x = X_REF.copy()
    x[3, 2] = -0.001
    rc, e, g, H = O.tet_elastic(X_REF, x, 1e5, 0.4)
    assert rc != 0 and e == math.inf


def test_projected_elastic_hessian_matches_eigh_projection():
    # 9x9 projection inside the oracle, compared through numpy's eigensolver
    rng = np.random.default_rng(3)
    x = X_REF + rng.normal(scale=3e-3, size=(4, 3))
    x[3] = X_REF[3] * [1, 1, 0.25] + [0.004, 0.001, 0]  # strongly compressed: indefinite Hessian
    rc, e, g, H = O.tet_elastic(X_REF, x, 1e5, 0.4, project=False)
    rc, e, g, Hp = O.tet_elastic(X_REF, x, 1e5, 0.4, project=True)
    assert rc == 0
    assert np.linalg.eigvalsh(H).min() < -1e-6 * np.abs(H).max()  # the case is really indefinite
    assert np.linalg.eigvalsh(Hp).min() > -1e-10 * np.abs(Hp).max()


# ---------------------------------------------------------------------------
# PSD projection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 9, 12])
def test_psd_projection_vs_eigh(n):
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    A = A + A.T
    P = O.psd_project(A)
    w, V = np.linalg.eigh(A)
    ref = (V * np.maximum(w, 0)) @ V.T
    assert np.allclose(P, ref, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(P).min() > -1e-12 * np.abs(A).max()
    assert np.allclose(O.psd_project(P), P, atol=1e-12 * np.abs(A).max())  # idempotent
    B = rng.normal(size=(n, n))
    B = B @ B.T
    assert np.allclose(O.psd_project(B), B, atol=1e-12 * np.abs(B).max())  # identity on PSD


# ---------------------------------------------------------------------------
# additive CCD
# ---------------------------------------------------------------------------
def _path_min_dist(kind, x, p, t_hi, n=10000):
    ts = np.linspace(0, t_hi, n)
    f = O.pt_classify if kind == 0 else O.ee_classify
    return min(f(x + t * p)[1] for t in ts)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("seed", range(8))
def test_accd_conservative(kind, seed):
    rng = np.random.default_rng(500 + seed + 20 * kind)
    x = rng.uniform(-1, 1, (4, 3))
    p = rng.uniform(-2, 2, (4, 3))
    a = O.accd(kind, x, p)
    assert 0 < a <= 1
    assert _path_min_dist(kind, x, p, a, 2000) > 0
    if a < 1:
        f = O.pt_classify if kind == 0 else O.ee_classify
        d0 = math.sqrt(f(x)[1])
        assert math.sqrt(f(x + a * p)[1]) <= 0.1 * d0 * (1 + 1e-9)


def test_accd_point_to_plane_closed_form():
    tri = np.array([[-1, -1, 0], [2, -1, 0], [-1, 2, 0]], float)
    x = np.vstack([[0.1, 0.1, 0.5], tri])
    p = np.zeros((4, 3))
    p[0, 2] = -1.0  # reaches the plane at t* = 0.5
    a = O.accd(0, x, p)
    assert 0.9 * 0.5 - 1e-12 <= a <= 0.5
    p[0, 2] = -0.2  # never reaches it
    assert O.accd(0, x, p) == 1.0


# ---------------------------------------------------------------------------
# scene-level pins
# ---------------------------------------------------------------------------
def test_lumped_mass_and_surface():
    sc = S.soft_cube_drop()
    s = O.Scene(sc)
    m = s.mass()
    V = sc["rest_pos"]  # volume of the jittered cube from the tets
    x = V[sc["tets"]]
    vol = np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 2)).sum() / 6
    assert m.sum() == pytest.approx(1000.0 * vol, rel=1e-13)
    t, e, v = s.surface()
    # 5x5 cells per face, 2 triangles each, 6 faces + 2 ground triangles; Euler: V - E + F = 2 per closed surface
    assert len(t) == 6 * 25 * 2 + 2
    nv_cube = len(set(t[:-2].ravel()))
    ne_cube = len([1 for a, b in e if a < 216 and b < 216])
    assert nv_cube - ne_cube + 300 == 2


def _brute_candidates(sc, s, x, p=None):
    t, e, v = s.surface()
    kin = sc["kin_group"] >= 0
    dh = sc["dhat"]

    def box(ids):
        pts = x[ids]
        if p is not None:
            pts = np.concatenate([pts, x[ids] + p[ids]], 0)
        return pts.min(0) - dh, pts.max(0) + dh

    out = set()
    for vi in v:
        blo, bhi = box([vi])
        for tri in t:
            if vi in tri or (kin[vi] and kin[tri].all()):
                continue
            lo, hi = box(list(tri))
            if np.all(blo <= hi) and np.all(lo <= bhi):
                out.add((0, vi, *tri))
    for i in range(len(e)):
        for j in range(i + 1, len(e)):
            a, b = e[i], e[j]
            if len(set(a) & set(b)) or (kin[a].all() and kin[b].all()):
                continue
            lo1, hi1 = box(list(a))
            lo2, hi2 = box(list(b))
            if np.all(lo1 <= hi2) and np.all(lo2 <= hi1):
                out.add((1, *a, *b))
    return out


def test_candidates_match_brute_force_on_tiny_scene():
    sc = S.two_tets(gap=0.0008)
    s = O.Scene(sc)
    x = sc["rest_pos"]
    got = {tuple(r) for r in s.candidates(x)}
    assert got == _brute_candidates(sc, s, x)
    rng = np.random.default_rng(0)
    p = rng.normal(scale=2e-3, size=x.shape)
    got = {tuple(r) for r in s.candidates(x, p)}
    assert got == _brute_candidates(sc, s, x, p)
    # every pair closer than dhat is a candidate and is active
    act, d2 = s.active(x)
    assert len(act) > 0 and np.all(d2 < sc["dhat"] ** 2)
    for row in act:
        assert tuple(row[:5]) in got


def test_active_set_is_exactly_pairs_within_dhat():
    sc = S.two_tets(gap=0.0006)
    s = O.Scene(sc)
    x = sc["rest_pos"]
    t, e, v = s.surface()
    act, d2 = s.active(x)
    got = {tuple(r[:5]) for r in act}
    ref = set()
    for vi in v:
        for tri in t:
            if vi in tri:
                continue
            if _pt_sampled(x[[vi, *tri]], 200) < sc["dhat"] ** 2 * (1 - 1e-3):
                ref.add((0, vi, *tri))
    for i in range(len(e)):
        for j in range(i + 1, len(e)):
            a, b = e[i], e[j]
            if len(set(a) & set(b)):
                continue
            if _ee_sampled(x[[*a, *b]], 200) < sc["dhat"] ** 2 * (1 - 1e-3):
                ref.add((1, *a, *b))
    assert ref <= got
    for r, dd in zip(act, d2):
        f = _pt_sampled if r[0] == 0 else _ee_sampled
        assert f(x[list(r[1:5])], 200) >= dd * (1 - 1e-9)


def test_scene_gradient_matches_fd_with_contact_and_friction():
    sc = S.block_on_incline(20.0, gap_frac=0.6, E=1e5)
    s = O.Scene(sc, linear_solver=1)
    s.step(1)  # builds a lagged friction set at the next step
    x0 = s.begin_step()
    fr = s.friction_pairs()
    assert len(fr[0]) > 0
    rng = np.random.default_rng(2)
    x = x0 + rng.normal(scale=2e-5, size=x0.shape) * (sc["kin_group"] < 0)[:, None]
    g, gabs = s.gradient(x)
    free = np.where(sc["kin_group"] < 0)[0]
    h = 1e-9
    for vi in free[:: max(1, len(free) // 6)]:
        for k in range(3):
            e = np.zeros_like(x)
            e[vi, k] = h
            fd = (s.energy(x + e) - s.energy(x - e)) / (2 * h)
            assert g[vi, k] == pytest.approx(fd, rel=1e-4, abs=1e-6 * gabs[vi, k])


def test_scene_hessian_is_fd_of_gradient_at_rest():
    sc = S.free_block(cells=1, gravity=(0, 0, 0))
    s = O.Scene(sc, linear_solver=1)
    x0 = s.begin_step()
    H = s.hessian_dense(x0)
    n = x0.size
    fH = np.zeros((n, n))
    h = 1e-8
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fH[:, i] = ((s.gradient((x0.reshape(-1) + e).reshape(-1, 3))[0] -
                     s.gradient((x0.reshape(-1) - e).reshape(-1, 3))[0]).reshape(-1)) / (2 * h)
    assert np.allclose(H, fH, rtol=1e-5, atol=1e-6 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() > 0


def test_pcg_matches_dense_solve():
    sc = S.soft_cube_drop(cells=2, edge=0.04)
    a = O.Scene(sc, pcg_rel_tol=1e-12)
    b = O.Scene(sc, linear_solver=1)
    xa, xb = a.begin_step(), b.begin_step()
    xa = xa + np.random.default_rng(1).normal(scale=1e-4, size=xa.shape) * (sc["kin_group"] < 0)[:, None]
    pa, it = a.newton_dir(xa)
    pb, _ = b.newton_dir(xa)
    assert it > 0
    assert np.allclose(pa, pb, rtol=1e-8, atol=1e-10 * np.abs(pb).max())


# ---------------------------------------------------------------------------
# physics cases with exact answers
# ---------------------------------------------------------------------------
def test_free_fall_matches_implicit_euler_closed_form():
    sc = S.free_block(cells=1)
    s = O.Scene(sc, linear_solver=1)
    x0 = sc["rest_pos"].copy()
    g = np.array([0, 0, -9.81])
    h = sc["dt"]
    for n in range(1, 6):
        rc, info = s.step(1)
        assert rc == 0
        pos, vel = s.state()
        ref = x0 + h * h * g * n * (n + 1) / 2
        assert np.allclose(pos, ref, atol=1e-12)
        assert np.allclose(vel, n * h * g, atol=1e-10)
        assert info["newton_iters"] <= 2


def test_momentum_conserved_without_gravity_or_contact():
    sc = S.free_block(cells=2, gravity=(0, 0, 0), vel=(0.3, -0.1, 0.2))
    s = O.Scene(sc)
    m = s.mass()
    p0 = (m[:, None] * sc["init_vel"]).sum(0)
    for _ in range(5):
        assert s.step(1)[0] == 0
    pos, vel = s.state()
    assert np.allclose((m[:, None] * vel).sum(0), p0, rtol=1e-9, atol=1e-12)


@pytest.mark.slow
def test_cube_drop_invariants_and_resting_force_balance():
    """Soft cube drop: zero penetration (Table I D1 = 0), J > 0, rest gap ~ dhat, sum of contact forces = weight."""
    sc = S.soft_cube_drop()
    s = O.Scene(sc)
    m = s.mass()
    W = m.sum() * 9.81
    for k in range(40):
        rc, info = s.step(1)
        assert rc == 0
        assert info["min_dist_last"] > 0
    pos, vel = s.state()
    assert np.abs(vel[sc["kin_group"] < 0]).max() < 1e-3
    gap = pos[sc["kin_group"] < 0, 2].min()
    assert 0.5 * sc["dhat"] < gap < sc["dhat"]
    s.begin_step()
    v, lam, nrm, w = s.friction_pairs()
    # contact force on the body: lambda along the normal pointing from the ground to the body
    fz = 0.0
    for vv, l, n, ww in zip(v, lam, nrm, w):
        body_side = [i for i in range(4) if sc["kin_group"][vv[i]] < 0]
        sgn = np.sign(sum(ww[i] for i in body_side))
        fz += l * n[2] * sgn
    assert fz == pytest.approx(W, rel=2e-3)
    _, _, cau, vm = s.state(stress=True)
    assert np.all(np.isfinite(vm)) and vm.max() > 0


@pytest.mark.slow
@pytest.mark.parametrize("theta,sticks", [(15.0, True), (45.0, False)])
def test_incline_friction(theta, sticks):
    mu = 0.5
    sc = S.block_on_incline(theta, mu=mu)
    s = O.Scene(sc)
    for _ in range(12):
        assert s.step(1)[0] == 0
    pos0, vel0 = s.state()
    n2 = 10
    for _ in range(n2):
        assert s.step(1)[0] == 0
    pos1, vel1 = s.state()
    free = sc["kin_group"] < 0
    h = sc["dt"]
    if sticks:
        slip = np.abs(pos1[free, 0] - pos0[free, 0]).max() / n2
        assert slip <= sc["eps_v"] * h
    else:
        a = (vel1[free, 0].mean() - vel0[free, 0].mean()) / (n2 * h)
        th = math.radians(theta)
        assert a == pytest.approx(9.81 * (math.sin(th) - mu * math.cos(th)), rel=0.05)


def test_line_search_decreases_energy():
    sc = S.soft_cube_drop(cells=2, edge=0.04, height=0.0012)
    s = O.Scene(sc)
    for _ in range(3):
        s.step(1)
    x = s.begin_step()
    for _ in range(3):
        p, _ = s.newton_dir(x)
        a = s.ccd_bound(x, p)
        e0 = s.energy(x)
        while s.energy(x + a * p) > e0:
            a /= 2
        x = x + a * p
        assert s.energy(x) <= e0


def test_rejects_bad_input():
    sc = S.soft_cube_drop(cells=2, edge=0.04)
    bad = dict(sc)
    bad["tets"] = sc["tets"][:, [1, 0, 2, 3]].copy()
    with pytest.raises(O.OracleError) as ei:
        O.Scene(bad)
    assert ei.value.code == -2
    bad = dict(sc)
    rp = sc["rest_pos"].copy()
    bad["init_pos"] = rp.copy()
    bad["init_pos"][: len(rp) - 4, 2] -= 0.03  # the cube straddles the ground plane
    with pytest.raises(O.OracleError) as ei:
        O.Scene(bad)
    assert ei.value.code == -3
    bad = dict(sc)
    bad["dt"] = 0.0
    with pytest.raises(O.OracleError) as ei:
        O.Scene(bad)
    assert ei.value.code == -1


@pytest.mark.parametrize("seed", range(4))
def test_mollified_ee_barrier_fd(seed):
    """Near-parallel edges: the mollifier is active (energy differs from the unmollified one)."""
    rng = np.random.default_rng(900 + seed)
    a0 = rng.uniform(-1e-3, 1e-3, 3)
    ea = np.array([0.01, 0.0, 0.0])
    eb = np.array([0.008, 0.00005 * (seed + 1), 0.00002])
    b0 = a0 + np.array([0.001, -0.0002, 0.0006])
    x = np.stack([a0, a0 + ea, b0, b0 + eb])
    t, d2 = O.ee_classify(x)
    assert 0 < d2 < 1e-6
    eps_x = 1e-3 * (ea @ ea) * (eb @ eb)
    c = np.sum(np.cross(ea, eb) ** 2)
    assert c < eps_x
    e, g, H = O.pair_barrier(1, t, x, 1e-3, 3e6, eps_x)
    e0 = O.pair_barrier(1, t, x, 1e-3, 3e6, 0.0)[0]
    q = c / eps_x
    assert e == pytest.approx(e0 * q * (2 - q), rel=1e-12)
    x0 = x.reshape(-1)
    h = 1e-9
    fg = _fd_grad(lambda y: O.pair_barrier(1, t, y.reshape(4, 3), 1e-3, 3e6, eps_x)[0], x0, h)
    assert np.allclose(g, fg, rtol=1e-5, atol=1e-6 * np.abs(g).max())
    fH = np.stack([_fd_grad(lambda y, i=i: O.pair_barrier(1, t, y.reshape(4, 3), 1e-3, 3e6, eps_x)[1][i], x0, h)
                   for i in range(12)])
    assert np.allclose(H, fH, rtol=1e-4, atol=1e-5 * np.abs(H).max())


def test_augmented_lagrangian_dirichlet_press():
    """A plate prescribed to move 3 mm per step onto a block 1.5 mm below it: the direct move would
    penetrate, so the kinematic vertices are driven by the augmented Lagrangian and snapped onto their
    targets; every step ends with the plate exactly on target, no intersection and no inversion."""
    sc = S.press_block(steps=3)
    o = O.Scene(sc)
    kin = sc["kin_group"]
    X = sc["rest_pos"]
    dt = sc["dt"]
    for k in range(3):
        rc, info = o.step(1)
        assert rc == 0, info
        assert info["min_dist_last"] > 0
        pos, vel = o.state()
        target = X[kin == 1, 2] - 0.3 * dt * (k + 1)
        assert np.array_equal(pos[kin == 1, 2], target)
        assert pos[kin < 0, 2].max() < target.min()
        x = pos[sc["tets"]]
        assert np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 2)).min() > 0
