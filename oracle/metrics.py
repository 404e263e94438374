"""Grasp-quality metrics D1 / D2 of Sec. IV-C, Eq. (2)-(3) -- plain numpy reference (test
infrastructure only: the tests, the smoke check and the benchmark's CPU-baseline leg may use it;
the library never does).

The manipuland's signed distance field d_o is taken from its closed, outward-oriented boundary
triangle mesh at the current positions: |d_o(p)| is the Euclidean distance from p to the nearest
surface triangle, positive when p lies inside the manipuland (penetration), negative outside.  Inside
is decided by the generalised winding number (sum of the solid angles of the oriented triangles seen
from p, over 4 pi): 1 inside a closed outward-oriented surface, 0 outside.  Over the sample set S_h on
the gripper's surface,

    D1 = max(0, max_{p in S_h} d_o(p)),      D2 = |max_{p in S_h} d_o(p)|,

so with no contact D1 = 0 and D2 is the gripper-manipuland gap; with penetration both equal the
penetration depth (Fig. 6 of the paper).

Everything here is the definition written out: distance to a triangle as the least of the distance to
its plane (when the foot of the perpendicular falls inside) and the distances to its three edges as
segments; solid angle by the formula of Van Oosterom and Strackee (1983).
"""
from __future__ import annotations

import numpy as np


def point_segment_distance(p, a, b):
    """Distance from points p [n,3] to segments (a, b) [n,3] (broadcast)."""
    e = b - a
    ee = np.sum(e * e, -1)
    t = np.where(ee > 0, np.sum((p - a) * e, -1) / np.where(ee > 0, ee, 1.0), 0.0)
    t = np.clip(t, 0.0, 1.0)
    q = a + t[..., None] * e
    return np.sqrt(np.sum((p - q) ** 2, -1))


def point_triangle_distance(p, t0, t1, t2):
    """Distance from points p to triangles (t0, t1, t2) (broadcast): the plane distance if the
    perpendicular foot lies in the triangle, else the least distance to the three edges."""
    n = np.cross(t1 - t0, t2 - t0)
    nn = np.sum(n * n, -1)
    h = np.sum((p - t0) * n, -1) / np.sqrt(nn)
    foot = p - (h / np.sqrt(nn))[..., None] * n
    # barycentric sign test of the foot: the three sub-triangle normals point along n
    s0 = np.sum(np.cross(t1 - foot, t2 - foot) * n, -1)
    s1 = np.sum(np.cross(t2 - foot, t0 - foot) * n, -1)
    s2 = np.sum(np.cross(t0 - foot, t1 - foot) * n, -1)
    inside = (s0 >= 0) & (s1 >= 0) & (s2 >= 0)
    edge = np.minimum(np.minimum(point_segment_distance(p, t0, t1), point_segment_distance(p, t1, t2)),
                      point_segment_distance(p, t2, t0))
    return np.where(inside, np.abs(h), edge)


def solid_angle(p, t0, t1, t2):
    """Signed solid angle of triangle (t0, t1, t2) seen from p (Van Oosterom-Strackee)."""
    a, b, c = t0 - p, t1 - p, t2 - p
    la, lb, lc = (np.sqrt(np.sum(v * v, -1)) for v in (a, b, c))
    num = np.sum(a * np.cross(b, c), -1)
    den = la * lb * lc + np.sum(a * b, -1) * lc + np.sum(a * c, -1) * lb + np.sum(b * c, -1) * la
    return 2.0 * np.arctan2(num, den)


def winding_number(points, verts, tris):
    """Generalised winding number of the oriented triangle mesh (verts, tris) at each point."""
    t0, t1, t2 = (verts[tris[:, k]] for k in range(3))
    out = np.empty(len(points))
    for i, p in enumerate(points):
        out[i] = solid_angle(p[None, :], t0, t1, t2).sum() / (4.0 * np.pi)
    return out


def signed_distance(points, verts, tris):
    """d_o at each point: distance to the nearest triangle, + inside (winding number > 1/2), - outside."""
    t0, t1, t2 = (verts[tris[:, k]] for k in range(3))
    d = np.empty(len(points))
    for i, p in enumerate(points):
        d[i] = point_triangle_distance(p[None, :], t0, t1, t2).min()
    inside = winding_number(points, verts, tris) > 0.5
    return np.where(inside, d, -d)


def sample_points(verts, hand_tris, sample_tri, sample_uv):
    """Sample positions p = (1-u-v) x0 + u x1 + v x2 on the listed hand triangles."""
    tri = hand_tris[sample_tri]
    u, v = sample_uv[:, 0:1], sample_uv[:, 1:2]
    return (1.0 - u - v) * verts[tri[:, 0]] + u * verts[tri[:, 1]] + v * verts[tri[:, 2]]


def grasp_metrics(verts, obj_tris, hand_tris, sample_tri, sample_uv):
    """(D1, D2, d_o at every sample) for positions verts [n,3] (Eq. (2)-(3))."""
    pts = sample_points(verts, hand_tris, sample_tri, sample_uv)
    d = signed_distance(pts, verts, obj_tris)
    m = float(d.max())
    return max(0.0, m), abs(m), d
