"""CPU pins of the oracle's grasp-quality metrics (Sec. IV-C, Eq. (2)-(3); oracle/metrics.py):

* signed distance to a triangulated box against the box's closed-form SDF (inside: distance to the
  nearest face; outside: Euclidean distance to the box, negative);
* point-triangle distance against dense sampling of the triangle;
* winding number 1 inside / 0 outside a voxel-tet body's boundary (scenes.body_surface), whose
  orientation the divergence theorem pins (sum of face centroid . area normal / 3 = volume);
* D1 / D2 as Fig. 6 illustrates them: no contact -> D1 = 0, D2 = the gap; penetration by delta ->
  D1 = D2 = delta.
"""
import numpy as np
import pytest

from oracle import metrics as M
from paper_2503_05020_amd import scenes as S


def _box_mesh(lo, hi):
    """The 12 outward triangles of the axis-aligned box [lo, hi]."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    v = np.array([[lo[0] if i & 1 == 0 else hi[0], lo[1] if i & 2 == 0 else hi[1], lo[2] if i & 4 == 0 else hi[2]]
                  for i in range(8)])
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    tris = []
    for a, b, c, d in quads:
        tris += [(a, b, c), (a, c, d)]
    tris = np.array(tris)
    # orient outward
    cen = 0.5 * (lo + hi)
    for t in tris:
        n = np.cross(v[t[1]] - v[t[0]], v[t[2]] - v[t[0]])
        if np.dot(n, v[t[0]] - cen) < 0:
            t[1], t[2] = t[2], t[1]
    return v, tris


def _box_sdf(p, lo, hi):
    lo, hi = np.asarray(lo), np.asarray(hi)
    out = np.maximum(np.maximum(lo - p, p - hi), 0.0)
    outside = np.linalg.norm(out, axis=1)
    inside = np.minimum((p - lo).min(1), (hi - p).min(1))
    return np.where((out > 0).any(1), -outside, inside)


def test_box_signed_distance_closed_form():
    lo, hi = [0.0, 0.0, 0.0], [1.0, 0.5, 2.0]
    v, tris = _box_mesh(lo, hi)
    rng = np.random.default_rng(0)
    p = rng.uniform([-0.7, -0.7, -0.7], [1.7, 1.2, 2.7], (400, 3))
    d = M.signed_distance(p, v, tris)
    ref = _box_sdf(p, lo, hi)
    assert np.abs(d - ref).max() < 1e-12
    assert (d > 0).sum() > 20 and (d < 0).sum() > 20


def test_point_triangle_distance_against_dense_sampling():
    rng = np.random.default_rng(1)
    g = np.linspace(0, 1, 401)
    U, V = np.meshgrid(g, g)
    keep = U + V <= 1
    U, V = U[keep], V[keep]
    for _ in range(30):
        t = rng.uniform(-1, 1, (3, 3))
        p = rng.uniform(-1.5, 1.5, 3)
        q = (1 - U - V)[:, None] * t[0] + U[:, None] * t[1] + V[:, None] * t[2]
        dense = np.linalg.norm(q - p, axis=1).min()
        d = float(M.point_triangle_distance(p[None], t[0][None], t[1][None], t[2][None])[0])
        h = np.linalg.norm(t - t.mean(0), axis=1).max() * 2.0 / 400  # grid spacing on the triangle
        assert d <= dense + 1e-12
        assert d >= dense - h


def test_winding_number_and_orientation_of_a_voxel_body():
    sc = S.soft_cube_drop(cells=3, edge=0.06, height=0.01)
    tris = S.body_surface(sc, 0)
    X = sc["rest_pos"]
    # divergence theorem: V = 1/3 sum over faces of centroid . (area normal)
    c = X[tris].mean(1)
    n = 0.5 * np.cross(X[tris[:, 1]] - X[tris[:, 0]], X[tris[:, 2]] - X[tris[:, 0]])
    vol = np.sum(c * n) / 3.0
    tets = sc["tets"]
    tv = np.abs(np.linalg.det(np.stack([X[tets[:, k]] - X[tets[:, 0]] for k in (1, 2, 3)], 2))).sum() / 6.0
    assert vol == pytest.approx(tv, rel=1e-12)
    lo, hi = X[sc["kin_group"] < 0].min(0), X[sc["kin_group"] < 0].max(0)
    rng = np.random.default_rng(2)
    inner = rng.uniform(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo), (20, 3))
    outer = hi + rng.uniform(0.01, 0.05, (20, 3))
    assert np.abs(M.winding_number(inner, X, tris) - 1.0).max() < 1e-9
    assert np.abs(M.winding_number(outer, X, tris)).max() < 1e-9


def test_d1_d2_as_in_fig6():
    """A flat 'finger' sampled above the box: with a gap g, D1 = 0 and D2 = g; pushed in by delta,
    D1 = D2 = delta (the deepest sample)."""
    v, tris = _box_mesh([0, 0, 0], [1, 1, 1])
    rng = np.random.default_rng(3)
    # finger: one triangle pair over the top face's centre region, sampled densely
    f = np.array([[0.3, 0.3, 0.0], [0.7, 0.3, 0.0], [0.7, 0.7, 0.0], [0.3, 0.7, 0.0]])
    ftris = np.array([[0, 1, 2], [0, 2, 3]]) + len(v)
    n = 200
    st = rng.integers(0, 2, n).astype(np.int32)
    uv = rng.uniform(size=(n, 2))
    flip = uv.sum(1) > 1
    uv[flip] = 1 - uv[flip]
    for z, d1, d2 in ((1.003, 0.0, 0.003), (0.996, 0.004, 0.004)):
        verts = np.concatenate([v, f + [0, 0, z]])
        D1, D2, d = M.grasp_metrics(verts, tris, ftris, st, uv)
        assert D1 == pytest.approx(d1, abs=1e-12)
        assert D2 == pytest.approx(d2, abs=1e-12)
