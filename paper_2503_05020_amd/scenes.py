"""Seeded synthetic grasp scenes (inputs only).

This module builds the meshes, materials and prescribed motions that both the
GPU library and the CPU oracle consume.  It holds none of the method's
arithmetic: no energies, distances, derivatives or solver steps -- only
geometry construction (voxel grids split into tetrahedra), random draws and
rigid motion schedules.

The paper's workloads are grasp validations of TetWild meshes from the
DexGraspNet / PartNet-Mobility sets (Sec. III-B) with the solver constants of
Sec. III-D (dt = 0.01 s, kappa = 3e6 kg/s^2, dhat = 1e-3 m, eps_v = 1e-3 m/s).
Those assets are not available, so voxel-tet scenes with the same sizes and
material ranges stand in for them.

Every scene is a plain dict of numpy arrays and scalars:

  rest_pos  [nv,3] f64   rest positions (also the initial positions)
  init_vel  [nv,3] f64   initial velocities (zeros)
  tets      [nt,4] i32   positively oriented tetrahedra
  E, nu, rho [nt]  f64   per-tet material
  tris      [nf,3] i32   kinematic-only surface triangles (ground, rigid links)
  kin_group [nv]   i32   -1 = free, g >= 0 = driven by motion group g
  motion    [S,G,12] f64 row-major 3x4 rigid transforms applied to rest_pos
  gravity   [S,3]  f64   gravity schedule (step n uses row min(n, S-1))
  dt, dhat, kappa, mu, eps_v, newton_tol, newton_max_iter
  env_bbox_diag          diagonal of the free vertices' rest bounding box
"""
from __future__ import annotations

import itertools
import math

import numpy as np

try:  # scipy's labelling keeps the largest face-connected voxel component
    from scipy import ndimage as _ndi
except Exception:  # pragma: no cover - scipy is present in this image
    _ndi = None

IDENTITY12 = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.float64)

DEFAULT_PARAMS = dict(dt=0.01, dhat=1e-3, kappa=3e6, mu=0.5, eps_v=1e-3,
                      newton_tol=1e-5, newton_max_iter=100)


# --------------------------------------------------------------------------
# voxel grids -> tetrahedra
# --------------------------------------------------------------------------
def _largest_component(mask: np.ndarray) -> np.ndarray:
    if _ndi is None or not mask.any():
        return mask
    lab, n = _ndi.label(mask)  # default structure = face (6-) connectivity
    if n <= 1:
        return mask
    counts = np.bincount(lab.ravel())
    counts[0] = 0
    return lab == int(np.argmax(counts))


# The six Kuhn (Freudenthal) tetrahedra of the unit cube around the
# (0,0,0)-(1,1,1) diagonal: one per permutation of the axes.  The split is
# conforming across neighbouring cells because every cell uses the same
# diagonal direction.
_UNIT = np.eye(3, dtype=np.int64)
_KUHN = []
for _perm in itertools.permutations(range(3)):
    _v0 = np.zeros(3, dtype=np.int64)
    _v1 = _v0 + _UNIT[_perm[0]]
    _v2 = _v1 + _UNIT[_perm[1]]
    _v3 = np.ones(3, dtype=np.int64)
    _KUHN.append((_v0, _v1, _v2, _v3))


def voxel_tet_mesh(mask: np.ndarray, h: float, origin) -> tuple[np.ndarray, np.ndarray]:
    """Tetrahedralise the cells of a boolean voxel mask (6 tets per cell).

    Returns (verts [nv,3] f64, tets [nt,4] i32).  Only the largest
    face-connected component is kept; unused grid nodes are dropped and tets
    are re-oriented so that det[x1-x0, x2-x0, x3-x0] > 0.
    """
    mask = _largest_component(np.asarray(mask, dtype=bool))
    nx, ny, nz = mask.shape
    cells = np.argwhere(mask)  # lexicographic (i, j, k) order
    if len(cells) == 0:
        return np.zeros((0, 3)), np.zeros((0, 4), dtype=np.int32)
    sy, sz = (ny + 1) * (nz + 1), nz + 1
    tets = []
    for corners in _KUHN:
        ids = [((cells + c) * np.array([sy, sz, 1])).sum(1) for c in corners]
        tets.append(np.stack(ids, 1))
    # interleave so that the six tets of one cell are consecutive
    tets = np.stack(tets, 1).reshape(-1, 4)
    used, inv = np.unique(tets, return_inverse=True)
    tets = inv.reshape(-1, 4).astype(np.int32)
    gi = used // sy
    gj = (used % sy) // sz
    gk = used % sz
    verts = np.stack([gi, gj, gk], 1).astype(np.float64) * h + np.asarray(origin, dtype=np.float64)
    _orient(verts, tets)
    return verts, tets


def _orient(verts: np.ndarray, tets: np.ndarray) -> None:
    x = verts[tets]
    d = np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 2))
    neg = d < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()


def _centres(n: int, h: float) -> np.ndarray:
    return (np.arange(n) + 0.5) * h - n * h / 2.0


def sphere_mask(radius: float, h: float) -> tuple[np.ndarray, np.ndarray]:
    n = max(1, int(math.ceil(2 * radius / h)))
    c = _centres(n, h)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return X * X + Y * Y + Z * Z < radius * radius, np.full(3, -n * h / 2.0)


def superquadric_mask(a, e1: float, e2: float, h: float):
    """Cells whose centre satisfies (|x/a1|^(2/e2) + |y/a2|^(2/e2))^(e2/e1) + |z/a3|^(2/e1) < 1."""
    ns = [max(1, int(math.ceil(2 * ai / h))) for ai in a]
    cs = [_centres(n, h) for n in ns]
    X, Y, Z = np.meshgrid(*cs, indexing="ij")
    f = (np.abs(X / a[0]) ** (2 / e2) + np.abs(Y / a[1]) ** (2 / e2)) ** (e2 / e1) + np.abs(Z / a[2]) ** (2 / e1)
    return f < 1.0, np.array([-n * h / 2.0 for n in ns])


def ellipsoid_mask(a, h: float):
    ns = [max(1, int(math.ceil(2 * ai / h))) for ai in a]
    cs = [_centres(n, h) for n in ns]
    X, Y, Z = np.meshgrid(*cs, indexing="ij")
    return (X / a[0]) ** 2 + (Y / a[1]) ** 2 + (Z / a[2]) ** 2 < 1.0, np.array([-n * h / 2.0 for n in ns])


def _tets_for_h(mask_fn, h):
    m, o = mask_fn(h)
    return int(_largest_component(m).sum()) * 6


def h_for_tet_target(mask_fn, target: int, h_lo: float, h_hi: float, rel: float = 0.05, iters: int = 60) -> float:
    """Bisect the voxel size so the tet count lands within +-rel of target."""
    best_h, best_err = h_hi, float("inf")
    lo, hi = h_lo, h_hi
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        n = _tets_for_h(mask_fn, mid)
        err = abs(n - target) / target
        if err < best_err:
            best_h, best_err = mid, err
        if err <= rel:
            return mid
        if n > target:
            lo = mid
        else:
            hi = mid
    return best_h


# --------------------------------------------------------------------------
# scene assembly helpers
# --------------------------------------------------------------------------
class _Builder:
    def __init__(self):
        self.verts, self.tets, self.E, self.nu, self.rho = [], [], [], [], []
        self.tris, self.kin, self.body = [], [], []
        self.nv = 0

    def add_body(self, verts, tets, E, nu, rho, kin=None):
        off = self.nv
        self.verts.append(np.asarray(verts, np.float64))
        self.tets.append(np.asarray(tets, np.int64) + off)
        nt = len(tets)
        self.E.append(np.broadcast_to(np.asarray(E, np.float64), (nt,)).copy())
        self.nu.append(np.broadcast_to(np.asarray(nu, np.float64), (nt,)).copy())
        self.rho.append(np.broadcast_to(np.asarray(rho, np.float64), (nt,)).copy())
        k = np.full(len(verts), -1, np.int32) if kin is None else np.asarray(kin, np.int32)
        self.kin.append(k)
        self.body.append(np.full(len(verts), len(self.body), np.int32))
        self.nv += len(verts)
        return off

    def add_kinematic_mesh(self, verts, tris, group):
        off = self.nv
        self.verts.append(np.asarray(verts, np.float64))
        self.tris.append(np.asarray(tris, np.int64) + off)
        self.kin.append(np.full(len(verts), group, np.int32))
        self.body.append(np.full(len(verts), len(self.body), np.int32))
        self.nv += len(verts)
        return off

    def build(self, motion, gravity, **params):
        p = dict(DEFAULT_PARAMS)
        p.update(params)
        verts = np.concatenate(self.verts, 0)
        kin = np.concatenate(self.kin, 0)
        free = kin < 0
        lo, hi = verts[free].min(0), verts[free].max(0)
        motion = np.asarray(motion, np.float64)
        gravity = np.asarray(gravity, np.float64).reshape(-1, 3)
        if len(gravity) == 1 and len(motion) > 1:
            gravity = np.repeat(gravity, len(motion), 0)
        assert len(gravity) == len(motion), "one gravity row per motion row"
        sc = dict(
            rest_pos=np.ascontiguousarray(verts),
            init_vel=np.zeros_like(verts),
            tets=np.ascontiguousarray(np.concatenate(self.tets, 0).astype(np.int32)) if self.tets else np.zeros((0, 4), np.int32),
            E=np.concatenate(self.E) if self.E else np.zeros(0),
            nu=np.concatenate(self.nu) if self.nu else np.zeros(0),
            rho=np.concatenate(self.rho) if self.rho else np.zeros(0),
            tris=np.ascontiguousarray(np.concatenate(self.tris, 0).astype(np.int32)) if self.tris else np.zeros((0, 3), np.int32),
            kin_group=np.ascontiguousarray(kin),
            motion=np.ascontiguousarray(np.asarray(motion, np.float64)),
            gravity=np.ascontiguousarray(np.asarray(gravity, np.float64)),
            env_bbox_diag=float(np.linalg.norm(hi - lo)),
            body=np.concatenate(self.body, 0),  # per vertex: the add_body / add_kinematic_mesh call it came from
        )
        sc.update(p)
        return sc


def body_surface(sc: dict, body: int) -> np.ndarray:
    """Boundary triangles [m,3] of one body of a scene (vertex ids of the scene), oriented outward at
    the rest positions: for a tet body its faces used by one tet only, each ordered so that the tet's
    fourth vertex lies behind it; for a kinematic mesh its own triangles."""
    vb = sc["body"]
    tets = np.asarray(sc["tets"])
    tets = tets[vb[tets[:, 0]] == body]
    if len(tets) == 0:
        tris = np.asarray(sc["tris"])
        return tris[vb[tris[:, 0]] == body].astype(np.int32)
    X = sc["rest_pos"]
    faces = {}
    for t in tets:
        for k in range(4):
            f = [t[j] for j in range(4) if j != k]
            key = tuple(sorted(f))
            if key in faces:
                faces[key] = None
            else:
                faces[key] = (f, t[k])
    out = []
    for v in faces.values():
        if v is None:
            continue
        f, opp = v
        n = np.cross(X[f[1]] - X[f[0]], X[f[2]] - X[f[0]])
        if np.dot(n, X[opp] - X[f[0]]) > 0:
            f = [f[0], f[2], f[1]]
        out.append(f)
    return np.array(out, np.int32)


def surface_samples(sc: dict, tris: np.ndarray, n: int, seed: int = 0):
    """n points on the triangles, uniform by rest area: (triangle index [n], barycentric (u, v) [n,2])."""
    rng = np.random.default_rng(seed)
    X = sc["rest_pos"]
    a = 0.5 * np.linalg.norm(np.cross(X[tris[:, 1]] - X[tris[:, 0]], X[tris[:, 2]] - X[tris[:, 0]]), axis=1)
    tri = rng.choice(len(tris), size=n, p=a / a.sum()).astype(np.int32)
    u, v = rng.uniform(size=n), rng.uniform(size=n)
    flip = u + v > 1.0
    u[flip], v[flip] = 1.0 - u[flip], 1.0 - v[flip]
    return tri, np.stack([u, v], 1)


def ground_plane(half: float = 0.5, z: float = 0.0):
    v = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float64)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int64)
    return v, t


def translation(t) -> np.ndarray:
    m = IDENTITY12.copy()
    m[3], m[7], m[11] = t
    return m


def static_motion(n_groups: int, n_steps: int = 1) -> np.ndarray:
    return np.tile(IDENTITY12, (n_steps, n_groups, 1))


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def soft_cube_drop(seed: int = 0, cells: int = 5, edge: float = 0.1, height: float = 0.01,
                   jitter: float = 1e-4, **params):
    """Soft cube (cells^3 voxels, 6 tets each) dropped onto a kinematic ground plane.

    5x5x5 cells of a 10 cm cube = 216 verts / 750 tets; bottom 1 cm above the
    plane; E = 1e5 Pa, nu = 0.4, rho = 1000; gravity 9.81; vertex jitter
    U[-1e-4, 1e-4] m applied before the rest shape is taken.
    """
    rng = np.random.default_rng(seed)
    h = edge / cells
    v, t = voxel_tet_mesh(np.ones((cells,) * 3, bool), h, (-edge / 2, -edge / 2, height))
    v = v + rng.uniform(-jitter, jitter, v.shape)
    b = _Builder()
    b.add_body(v, t, 1e5, 0.4, 1000.0)
    gv, gt = ground_plane()
    b.add_kinematic_mesh(gv, gt, 0)
    return b.build(static_motion(1), [[0.0, 0.0, -9.81]], **params)


def stacked_cubes(n: int, cells: int = 2, edge: float = 0.03, gap: float = 0.004, **params):
    """n soft cubes (cells^3 voxels each, E = 1e5 Pa, nu = 0.4, rho = 1000) stacked along z with
    `gap` between them and above a kinematic ground plane, each shifted 2 mm along x from the one
    below; gravity 9.81.  n separate bodies: a scene with several connected sets of free vertices."""
    b = _Builder()
    h = edge / cells
    for k in range(n):
        origin = (-edge / 2 + 0.002 * k, -edge / 2, gap + k * (edge + gap))
        v, t = voxel_tet_mesh(np.ones((cells,) * 3, bool), h, origin)
        b.add_body(v, t, 1e5, 0.4, 1000.0)
    gv, gt = ground_plane()
    b.add_kinematic_mesh(gv, gt, 0)
    return b.build(static_motion(1), [[0.0, 0.0, -9.81]], **params)


def pinned_column(cells: int = 3, h: float = 0.01, **params):
    """A soft voxel column (1 x 1 x cells cells) whose vertices are all held in place except the
    cells + 1 on one vertical edge: the only free vertices lie on a line (a body whose rotation
    about that line moves nothing).  Gravity 9.81."""
    v, t = voxel_tet_mesh(np.ones((1, 1, cells), bool), h, (0.0, 0.0, 0.005))
    line = (np.abs(v[:, 0] - v[:, 0].min()) < 1e-12) & (np.abs(v[:, 1] - v[:, 1].min()) < 1e-12)
    b = _Builder()
    b.add_body(v, t, 1e5, 0.4, 1000.0, kin=np.where(line, -1, 0))
    return b.build(static_motion(1), [[0.0, 0.0, -9.81]], **params)


def _slab(h: float = 0.004, cells=(2, 4, 10)):
    """Finger slab: cells along (closing, width, length) = 8 x 16 x 40 mm at 4 mm."""
    v, t = voxel_tet_mesh(np.ones(cells, bool), h, (0.0, 0.0, 0.0))
    return v, t


def _frame_from(approach, roll):
    a = np.asarray(approach, np.float64)
    a = a / np.linalg.norm(a)
    helper = np.array([1.0, 0, 0]) if abs(a[0]) < 0.9 else np.array([0, 1.0, 0])
    u0 = np.cross(a, helper)
    u0 /= np.linalg.norm(u0)
    w0 = np.cross(a, u0)
    u = math.cos(roll) * u0 + math.sin(roll) * w0
    w = np.cross(a, u)
    return u, w, a


def _add_gripper(b: _Builder, obj_verts, centre, u, w, a, gap=0.002, close_speed=0.01,
                 close_steps=60, lift_speed=0.02, lift_steps=40, dt=0.01, lift_dir=(0, 0, 1),
                 E=5e5, nu=0.45, rho=1000.0, first_group=0):
    """Two soft finger slabs on either side of the object along closing axis u.

    The slab's outer face (farthest from the object) is kinematic and follows
    a closing translation at close_speed, then a lift at lift_speed.
    """
    sv, st = _slab()
    sv = sv - np.array([0.0, 0.008, 0.02])  # centre in width and length
    rel = obj_verts - centre
    sup_hi = float((rel @ u).max())
    sup_lo = float((rel @ u).min())
    n_steps = close_steps + lift_steps + 1
    motions = np.zeros((n_steps, 2, 12))
    lift_dir = np.asarray(lift_dir, np.float64)
    for side, (sign, sup) in enumerate(((+1.0, sup_hi), (-1.0, sup_lo))):
        # local coords: x along +sign*u (0 at inner face), y along w, z along a
        x_local = sv[:, 0]
        off = sup + sign * gap
        world = (centre + np.outer(off + sign * x_local, u) + np.outer(sv[:, 1], w) + np.outer(sv[:, 2], a))
        kin = np.where(np.isclose(x_local, x_local.max()), first_group + side, -1).astype(np.int32)
        tets = st.copy()
        _orient(world, tets)  # the mirrored slab flips orientation
        b.add_body(world, tets, E, nu, rho, kin)
        for n in range(n_steps):
            nc = min(n, close_steps)
            nl = max(0, n - close_steps)
            disp = -sign * u * close_speed * dt * nc + lift_dir * lift_speed * dt * nl
            motions[n, side] = translation(disp)
    return motions


def parallel_jaw_sphere(seed: int = 0, radius: float = 0.03, h: float = 0.0044, tet_target=None, **params):
    """Two soft finger slabs squeeze a soft voxel sphere resting on a ground plane.

    Sphere r = 3 cm (~8k tets at h = 4.4 mm), E log-uniform [1e4, 1e6] Pa,
    nu U[0.3, 0.45]; fingers 40x16x8 mm, E = 5e5, nu = 0.45, closing 1 cm/s
    for 60 steps then lifting 2 cm/s for 40 steps.
    """
    rng = np.random.default_rng(seed)
    if tet_target is not None:
        h = h_for_tet_target(lambda hh: sphere_mask(radius, hh), tet_target, 0.5e-3, 0.02)
    m, origin = sphere_mask(radius, h)
    sv, stt = voxel_tet_mesh(m, h, origin)
    dhat = params.get("dhat", DEFAULT_PARAMS["dhat"])
    sv[:, 2] += -sv[:, 2].min() + 1.2 * dhat
    E = math.exp(rng.uniform(math.log(1e4), math.log(1e6)))
    nu = rng.uniform(0.3, 0.45)
    b = _Builder()
    b.add_body(sv, stt, E, nu, 1000.0)
    centre = np.array([0.0, 0.0, sv[:, 2].mean()])
    centre[0] = 0.5 * (sv[:, 0].min() + sv[:, 0].max())
    u, w, a = np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])
    fm = _add_gripper(b, sv, centre, u, w, a, first_group=1)
    gv, gt = ground_plane()
    b.add_kinematic_mesh(gv, gt, 0)
    motion = np.concatenate([np.tile(IDENTITY12, (fm.shape[0], 1, 1)), fm], 1)
    return b.build(motion, [[0.0, 0.0, -9.81]], **params)


def superquadric_grasp(seed: int, tet_median: float = 5000.0, sigma: float = 0.6,
                       clip=(1000, 20000), **params):
    """One environment of the batched workload: a soft superquadric held by the two-slab gripper.

    e1, e2 ~ U[0.3, 2]; half-axes U[2, 8] cm; tet count lognormal(median
    5k, sigma 0.6) clipped to [1k, 20k]; E log-U[1e4, 1e6]; nu U[0.3, 0.45];
    rho U[500, 1500]; mu U[0.3, 0.8]; approach direction uniform on the
    sphere with uniform roll; no ground; gravity off for the 60 closing
    steps, then -z.
    """
    rng = np.random.default_rng(seed)
    e1, e2 = rng.uniform(0.3, 2.0, 2)
    a = rng.uniform(0.02, 0.08, 3)
    target = int(np.clip(math.exp(rng.normal(math.log(tet_median), sigma)), *clip))
    E = math.exp(rng.uniform(math.log(1e4), math.log(1e6)))
    nu = rng.uniform(0.3, 0.45)
    rho = rng.uniform(500.0, 1500.0)
    mu = rng.uniform(0.3, 0.8)
    d = rng.normal(size=3)
    approach = d / np.linalg.norm(d)
    roll = rng.uniform(0.0, 2 * math.pi)
    fn = lambda hh: superquadric_mask(a, e1, e2, hh)
    h = h_for_tet_target(fn, target, 0.5e-3, 0.05)
    m, origin = fn(h)
    ov, ot = voxel_tet_mesh(m, h, origin)
    b = _Builder()
    b.add_body(ov, ot, E, nu, rho)
    centre = 0.5 * (ov.min(0) + ov.max(0))
    u, w, ax = _frame_from(approach, roll)
    fm = _add_gripper(b, ov, centre, u, w, ax, first_group=0)
    grav = np.zeros((fm.shape[0], 3))
    grav[60:, 2] = -9.81
    p = dict(params)
    p.setdefault("mu", mu)
    sc = b.build(fm, grav, **p)
    sc["tet_target"] = target
    sc["voxel_h"] = h
    return sc


def batched_superquadrics(n_envs: int = 256, first_seed: int = 0, **kw):
    return [superquadric_grasp(first_seed + i, **kw) for i in range(n_envs)]


def serving_requests(n: int = 2000, rate: float = 50.0, seed: int = 1, tet_median: float = 1e4,
                     sigma: float = 0.6, clip=(2000, 50000)):
    """Poisson arrival schedule of sphere-grasp requests (scenes built lazily by seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps)
    targets = np.clip(np.exp(rng.normal(math.log(tet_median), sigma, n)), *clip).astype(np.int64)
    seeds = rng.integers(0, 2**31 - 1, n)
    return [dict(arrival=float(t), tet_target=int(k), seed=int(s)) for t, k, s in zip(arrivals, targets, seeds)]


def serving_scene(req):
    return parallel_jaw_sphere(seed=req["seed"], tet_target=req["tet_target"])


def capsule_mesh(length: float, radius: float, around: int = 16):
    """Closed capsule surface: 8 rings of `around` vertices plus two poles.

    Rings: three on each hemisphere (polar angles 30, 60, 90 deg) and two on
    the cylinder at 1/3 and 2/3 of `length`; the axis runs from (0,0,0) to
    (0,0,length).  16 around gives 130 vertices and 256 triangles.
    """
    rings = []
    for phi in (30.0, 60.0, 90.0):  # bottom hemisphere, pole at z = -radius
        t = math.radians(phi)
        rings.append((-radius * math.cos(t), radius * math.sin(t)))
    rings += [(length / 3.0, radius), (2.0 * length / 3.0, radius)]
    for phi in (90.0, 120.0, 150.0):  # top hemisphere
        t = math.radians(phi)
        rings.append((length - radius * math.cos(t), radius * math.sin(t)))
    ang = 2.0 * math.pi * np.arange(around) / around
    v = [[0.0, 0.0, -radius]]
    for z, r in rings:
        v += [[r * math.cos(a), r * math.sin(a), z] for a in ang]
    v.append([0.0, 0.0, length + radius])
    v = np.array(v)
    top = len(v) - 1
    t = []
    for j in range(around):  # bottom cap, outward normals
        t.append([0, 1 + (j + 1) % around, 1 + j])
    for k in range(len(rings) - 1):
        a0, a1 = 1 + k * around, 1 + (k + 1) * around
        for j in range(around):
            j1 = (j + 1) % around
            t.append([a0 + j, a0 + j1, a1 + j1])
            t.append([a0 + j, a1 + j1, a1 + j])
    last = 1 + (len(rings) - 1) * around
    for j in range(around):
        t.append([top, last + j, last + (j + 1) % around])
    return v, np.array(t, np.int64)


def _rot_x(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rigid_hand_grasp(seed: int = 0, h: float = 2.08e-3, axes=(0.06, 0.04, 0.03), close_steps: int = 80,
                     lift_steps: int = 40, lift_speed: float = 0.05, closed_pose=(12.0, 8.0, 6.0, 4.0), **params):
    """A kinematic four-finger hand of 16 capsule links grasps a soft ellipsoid on the ground.

    Ellipsoid half-axes 6 x 4 x 3 cm (201k tets at h = 2.08 mm), E = 1e5,
    nu = 0.4, rho = 1000.  Fingers: two on each side of the y extent, at
    x = +-2.2 cm, hanging from 4.5 cm above the centre; links 45/35/25/20 mm
    long, radius 8 mm.  Joint angles (rotation about x, inward positive) go
    linearly from a seeded open pose (joint 0 at -15 deg, others 0, each
    +-10 deg) to the closed pose (default 12, 8, 6, 4 deg: the links press
    about 3 mm into the ellipsoid's rest shape) over `close_steps`
    steps, then the hand rises at `lift_speed` for `lift_steps` steps.
    dt = 5 ms, dhat = 0.5 mm, mu = 0.6.  Every link is its own kinematic group
    (0..15), the ground is group 16.  Links press into the object, so the
    prescribed moves need the augmented-Lagrangian mode.
    """
    p = dict(dt=0.005, dhat=5e-4, mu=0.6)
    p.update(params)
    dhat = p["dhat"]
    rng = np.random.default_rng(seed)
    m, origin = ellipsoid_mask(axes, h)
    ev, et = voxel_tet_mesh(m, h, origin)
    ev[:, 2] += -ev[:, 2].min() + 1.2 * dhat
    cz = 0.5 * (ev[:, 2].min() + ev[:, 2].max())
    b = _Builder()
    b.add_body(ev, et, 1e5, 0.4, 1000.0)
    lengths, radius = (0.045, 0.035, 0.025, 0.020), 0.008
    open_pose = np.array([-15.0, 0.0, 0.0, 0.0])
    closed_pose = np.array(closed_pose, dtype=float)
    n_rows = close_steps + lift_steps + 1
    motion = np.tile(IDENTITY12, (n_rows, 17, 1))
    group = 0
    for side in (-1.0, 1.0):
        for xf in (-0.022, 0.022):
            th_open = np.radians(open_pose + rng.uniform(-10.0, 10.0, 4))
            th_closed = np.radians(closed_pose)
            base = np.array([xf, side * (axes[1] + radius + 0.004), cz + 0.045])

            def chain(th):
                # joint positions and link rotations; a link's local +z maps to
                # (0, -side sin T, -cos T), T = the cumulative joint angle
                P, Rs, T = [base.copy()], [], 0.0
                for k in range(4):
                    T += th[k]
                    R = _rot_x(-side * T) @ np.diag([1.0, -1.0, -1.0])  # local +z -> straight down at T = 0
                    Rs.append(R)
                    P.append(P[-1] + lengths[k] * R[:, 2])
                return P, Rs

            P0, R0 = chain(th_open)
            for k in range(4):
                cv, ct = capsule_mesh(lengths[k], radius)
                world = cv @ R0[k].T + P0[k]
                b.add_kinematic_mesh(world, ct, group + k)
            for n in range(n_rows):
                f = min(n, close_steps) / close_steps
                Pn, Rn = chain(th_open + (th_closed - th_open) * f)
                lift = np.array([0.0, 0.0, lift_speed * p["dt"] * max(0, n - close_steps)])
                for k in range(4):
                    R = Rn[k] @ R0[k].T
                    t = Pn[k] + lift - R @ P0[k]
                    motion[n, group + k] = np.concatenate([np.c_[R, t]]).reshape(-1)
            group += 4
    gv, gt = ground_plane()
    b.add_kinematic_mesh(gv, gt, 16)
    return b.build(motion, [[0.0, 0.0, -9.81]], **p)


# --------------------------------------------------------------------------
# tiny fixtures
# --------------------------------------------------------------------------
def single_tet_on_ground(height: float = 0.005, size: float = 0.02, **params):
    v = np.array([[0, 0, 0], [size, 0, 0], [0, size, 0], [0, 0, size]], np.float64) + [0, 0, height]
    b = _Builder()
    b.add_body(v, np.array([[0, 1, 2, 3]]), 1e5, 0.4, 1000.0)
    gv, gt = ground_plane()
    b.add_kinematic_mesh(gv, gt, 0)
    return b.build(static_motion(1), [[0.0, 0.0, -9.81]], **params)


def two_tets(gap: float = 0.003, **params):
    v = np.array([[0, 0, 0], [0.02, 0, 0], [0, 0.02, 0], [0, 0, 0.02]], np.float64)
    w = v * [1, 1, -1] + [0.001, 0.002, -gap]
    b = _Builder()
    b.add_body(v, np.array([[0, 1, 2, 3]]), 1e5, 0.4, 1000.0)
    t2 = np.array([[0, 2, 1, 3]])
    b.add_body(w, t2, 1e5, 0.4, 1000.0)
    sc = b.build(static_motion(1), [[0.0, 0.0, 0.0]], **params)
    return sc


def free_block(cells: int = 2, edge: float = 0.02, gravity=(0.0, 0.0, -9.81), vel=(0.0, 0.0, 0.0), **params):
    v, t = voxel_tet_mesh(np.ones((cells,) * 3, bool), edge / cells, (0.0, 0.0, 0.5))
    b = _Builder()
    b.add_body(v, t, 1e5, 0.4, 1000.0)
    sc = b.build(static_motion(1), [list(gravity)], **params)
    sc["init_vel"] = np.tile(np.asarray(vel, np.float64), (len(v), 1))
    return sc


def block_on_incline(theta_deg: float, cells: int = 2, edge: float = 0.02, mu: float = 0.5,
                     E: float = 1e6, gap_frac: float = 1.5, **params):
    """A soft block resting on a kinematic plane tilted by theta about the y axis.

    Expressed in the plane's frame: the plane is z = 0 and gravity is tilted,
    so the block slides along +x when tan(theta) > mu.
    """
    dhat = params.get("dhat", DEFAULT_PARAMS["dhat"])
    v, t = voxel_tet_mesh(np.ones((cells,) * 3, bool), edge / cells, (-edge / 2, -edge / 2, gap_frac * dhat))
    b = _Builder()
    b.add_body(v, t, E, 0.4, 1000.0)
    gv, gt = ground_plane(0.5)
    b.add_kinematic_mesh(gv, gt, 0)
    th = math.radians(theta_deg)
    g = [9.81 * math.sin(th), 0.0, -9.81 * math.cos(th)]
    return b.build(static_motion(1), [g], mu=mu, **params)


def random_pt(rng, scale=1.0):
    return rng.uniform(-scale, scale, (4, 3))


def random_ee(rng, scale=1.0):
    return rng.uniform(-scale, scale, (4, 3))


def press_block(speed: float = 0.3, gap: float = 1.5e-3, cells: int = 2, edge: float = 0.02, steps: int = 8,
                E: float = 1e5, jitter: float = 0.05, seed: int = 0, **params):
    """A kinematic square plate pressed down onto a soft block resting on a ground plane.

    The plate starts `gap` above the block and moves down at `speed` for
    `steps` steps, then stops; at 0.3 m/s it covers 3 mm per step, more than
    the gap, so the prescribed move cannot be applied in one go.  The block's
    vertices are moved sideways by a seeded `jitter` (fraction of a cell):
    a perfectly symmetric block can twist either way under the press, and the
    branch taken would then be decided by rounding.
    """
    dhat = params.get("dhat", DEFAULT_PARAMS["dhat"])
    v, t = voxel_tet_mesh(np.ones((cells,) * 3, bool), edge / cells, (-edge / 2, -edge / 2, 1.2 * dhat))
    rng = np.random.default_rng(seed)
    v = v.copy()
    v[:, :2] += rng.uniform(-1.0, 1.0, (len(v), 2)) * jitter * edge / cells
    b = _Builder()
    b.add_body(v, t, E, 0.4, 1000.0)
    top = v[:, 2].max()
    hp = edge  # plate half-size: twice the block
    pv = np.array([[-hp, -hp, top + gap], [hp, -hp, top + gap], [hp, hp, top + gap], [-hp, hp, top + gap]])
    b.add_kinematic_mesh(pv, np.array([[0, 1, 2], [0, 2, 3]]), 1)
    gv, gt = ground_plane()
    b.add_kinematic_mesh(gv, gt, 0)
    dt = params.get("dt", DEFAULT_PARAMS["dt"])
    n = steps + 4
    motion = np.zeros((n, 2, 12))
    for k in range(n):
        motion[k, 0] = IDENTITY12
        motion[k, 1] = translation((0.0, 0.0, -speed * dt * min(k, steps)))
    return b.build(motion, [[0.0, 0.0, -9.81]], **params)
