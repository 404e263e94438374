"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It loads ``liboracle.so`` built from ``ipc_oracle.cpp``
by :func:`build`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "ipc_oracle.cpp")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Desc(C.Structure):
    _fields_ = [
        ("n_verts", C.c_int32), ("rest_pos", _dp), ("init_pos", _dp), ("init_vel", _dp),
        ("n_tets", C.c_int32), ("tets", _ip), ("E", _dp), ("nu", _dp), ("rho", _dp),
        ("n_tris", C.c_int32), ("tris", _ip), ("kin_group", _ip),
        ("n_groups", C.c_int32), ("n_motion_steps", C.c_int32), ("motion", _dp), ("gravity", _dp),
        ("dt", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double), ("mu", C.c_double),
        ("eps_v", C.c_double), ("newton_tol", C.c_double), ("newton_max_iter", C.c_int32),
        ("pcg_rel_tol", C.c_double), ("linear_solver", C.c_int32),
        ("newton_rel_tol", C.c_double), ("friction_iters", C.c_int32), ("inversion_filter", C.c_int32),
        ("adaptive_kappa", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("steps_done", C.c_int32), ("status", C.c_int32), ("fail_reason", C.c_int32),
        ("newton_iters", C.c_int32), ("max_newton_iters", C.c_int32), ("ls_halvings", C.c_int32),
        ("pcg_iters", C.c_int64), ("n_active_last", C.c_int64), ("min_dist_last", C.c_double),
        ("energy_last", C.c_double), ("kappa_last", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (FP contraction off)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-o", LIB_PATH + ".tmp", SRC]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.ipco_create.argtypes = [C.POINTER(Desc), C.POINTER(C.c_void_p)]
        L.ipco_destroy.argtypes = [C.c_void_p]
        L.ipco_destroy.restype = None
        L.ipco_last_error.restype = C.c_char_p
        L.ipco_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Info)]
        L.ipco_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.ipco_set_state.argtypes = [C.c_void_p, _dp, _dp, C.c_int32]
        L.ipco_get_step.argtypes = [C.c_void_p]
        L.ipco_surface_sizes.argtypes = [C.c_void_p, _ip]
        L.ipco_surface.argtypes = [C.c_void_p, _ip, _ip, _ip]
        L.ipco_mass.argtypes = [C.c_void_p, _dp]
        L.ipco_candidates.argtypes = [C.c_void_p, _dp, _dp, _ip, C.c_int64]
        L.ipco_candidates.restype = C.c_int64
        L.ipco_active.argtypes = [C.c_void_p, _dp, _ip, _dp, C.c_int64]
        L.ipco_active.restype = C.c_int64
        L.ipco_begin_step.argtypes = [C.c_void_p, _dp]
        L.ipco_energy.argtypes = [C.c_void_p, _dp]
        L.ipco_energy.restype = C.c_double
        L.ipco_gradient.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.ipco_hessian_dense.argtypes = [C.c_void_p, _dp, _dp]
        L.ipco_newton_dir.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_int64)]
        L.ipco_ccd_bound.argtypes = [C.c_void_p, _dp, _dp]
        L.ipco_ccd_bound.restype = C.c_double
        L.ipco_friction_pairs.argtypes = [C.c_void_p, _ip, _dp, _dp, _dp, C.c_int64]
        L.ipco_friction_pairs.restype = C.c_int64
        L.ipco_pt_classify.argtypes = [_dp, _dp]
        L.ipco_ee_classify.argtypes = [_dp, _dp]
        L.ipco_barrier_scalar.argtypes = [C.c_double, C.c_double, _dp]
        L.ipco_pair_barrier.argtypes = [C.c_int, C.c_int, _dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                        _dp, _dp, _dp]
        L.ipco_tet_elastic.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_int, _dp, _dp, _dp]
        L.ipco_psd_project.argtypes = [C.c_int, _dp]
        L.ipco_accd.argtypes = [C.c_int, _dp, _dp, C.c_double]
        L.ipco_accd.restype = C.c_double
        L.ipco_friction_f0.argtypes = [C.c_double, C.c_double, _dp]
        L.ipco_friction_elem.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.ipco_iter_log.argtypes = [C.c_void_p, _dp, C.c_int64]
        L.ipco_iter_log.restype = C.c_int64
        L.ipco_debug_ls_offset.argtypes = [C.c_void_p, C.c_double]
        L.ipco_tet_first_root.argtypes = [_dp, _dp, C.c_double, _dp]
        L.ipco_tet_first_root.restype = C.c_double
        L.ipco_inversion_bound.argtypes = [C.c_void_p, _dp, _dp]
        L.ipco_inversion_bound.restype = C.c_double
        L.ipco_kappa.argtypes = [C.c_void_p]
        L.ipco_kappa.restype = C.c_double
        L.ipco_contact_forces.argtypes = [C.c_void_p, _dp, _ip, C.c_int32, _dp]
        L.ipco_hold_group.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.ipco_set_gravity.argtypes = [C.c_void_p, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise OracleError(rc, lib().ipco_last_error().decode())
    return rc


class Scene:
    """One scene held by the oracle."""

    def __init__(self, sc: dict, pcg_rel_tol: float = 1e-8, linear_solver: int = 0, **overrides):
        p = dict(sc)
        p.update(overrides)
        self._keep = dict(
            rest=_f64(p["rest_pos"]).reshape(-1),
            init=_f64(p.get("init_pos", p["rest_pos"])).reshape(-1),
            vel=_f64(p.get("init_vel", np.zeros_like(p["rest_pos"]))).reshape(-1),
            tets=_i32(p["tets"]).reshape(-1), E=_f64(p["E"]), nu=_f64(p["nu"]), rho=_f64(p["rho"]),
            tris=_i32(p["tris"]).reshape(-1), kin=_i32(p["kin_group"]),
            motion=_f64(p["motion"]).reshape(-1), gravity=_f64(p["gravity"]).reshape(-1),
        )
        k = self._keep
        self.nv = len(k["kin"])
        self.nt = len(k["E"])
        motion = np.asarray(p["motion"])
        if motion.ndim != 3 or motion.shape[2] != 12 or np.asarray(p["gravity"]).reshape(-1, 3).shape[0] != motion.shape[0]:
            raise ValueError("motion must be [steps][groups][12] with one gravity row per step")
        d = Desc(self.nv, _d(k["rest"]), _d(k["init"]), _d(k["vel"]), self.nt, _i(k["tets"]), _d(k["E"]),
                 _d(k["nu"]), _d(k["rho"]), len(k["tris"]) // 3, _i(k["tris"]), _i(k["kin"]),
                 motion.shape[1], motion.shape[0], _d(k["motion"]), _d(k["gravity"]),
                 p["dt"], p["dhat"], p["kappa"], p["mu"], p["eps_v"], p["newton_tol"], int(p["newton_max_iter"]),
                 pcg_rel_tol, linear_solver, float(p.get("newton_rel_tol", 0.0)), int(p.get("friction_iters", 1)),
                 int(p.get("inversion_filter", 0)), int(p.get("adaptive_kappa", 0)))
        h = C.c_void_p()
        _check(lib().ipco_create(C.byref(d), C.byref(h)))
        self.h = h
        self.params = p

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.ipco_destroy(self.h)
            self.h = None

    def step(self, n=1):
        info = Info()
        rc = lib().ipco_step(self.h, n, C.byref(info))
        return rc, info.as_dict()

    def state(self, stress=False):
        pos = np.zeros((self.nv, 3))
        vel = np.zeros((self.nv, 3))
        cau = np.zeros((self.nt, 6)) if stress else None
        vm = np.zeros(self.nt) if stress else None
        _check(lib().ipco_get_state(self.h, _d(pos), _d(vel), _d(cau), _d(vm)))
        return (pos, vel, cau, vm) if stress else (pos, vel)

    def set_state(self, pos, vel, step):
        _check(lib().ipco_set_state(self.h, _d(_f64(pos)), _d(_f64(vel)), step))

    @property
    def step_index(self):
        return lib().ipco_get_step(self.h)

    def surface(self):
        n = np.zeros(3, np.int32)
        lib().ipco_surface_sizes(self.h, _i(n))
        t = np.zeros((n[0], 3), np.int32)
        e = np.zeros((n[1], 2), np.int32)
        v = np.zeros(n[2], np.int32)
        lib().ipco_surface(self.h, _i(t), _i(e), _i(v))
        return t, e, v

    def mass(self):
        m = np.zeros(self.nv)
        lib().ipco_mass(self.h, _d(m))
        return m

    def candidates(self, x, p=None):
        x = _f64(x)
        p = None if p is None else _f64(p)
        n = lib().ipco_candidates(self.h, _d(x), _d(p), None, 0)
        out = np.zeros((max(n, 1), 5), np.int32)
        lib().ipco_candidates(self.h, _d(x), _d(p), _i(out), n)
        return out[:n]

    def active(self, x):
        x = _f64(x)
        n = lib().ipco_active(self.h, _d(x), None, None, 0)
        out = np.zeros((max(n, 1), 6), np.int32)
        d2 = np.zeros(max(n, 1))
        lib().ipco_active(self.h, _d(x), _i(out), _d(d2), n)
        return out[:n], d2[:n]

    def begin_step(self):
        x0 = np.zeros((self.nv, 3))
        _check(lib().ipco_begin_step(self.h, _d(x0)))
        return x0

    def energy(self, x):
        return lib().ipco_energy(self.h, _d(_f64(x)))

    def gradient(self, x):
        g = np.zeros((self.nv, 3))
        ga = np.zeros((self.nv, 3))
        _check(lib().ipco_gradient(self.h, _d(_f64(x)), _d(g), _d(ga)))
        return g, ga

    def hessian_dense(self, x):
        H = np.zeros((3 * self.nv, 3 * self.nv))
        _check(lib().ipco_hessian_dense(self.h, _d(_f64(x)), _d(H)))
        return H

    def newton_dir(self, x):
        p = np.zeros((self.nv, 3))
        it = C.c_int64()
        _check(lib().ipco_newton_dir(self.h, _d(_f64(x)), _d(p), C.byref(it)))
        return p, it.value

    def ccd_bound(self, x, p):
        return lib().ipco_ccd_bound(self.h, _d(_f64(x)), _d(_f64(p)))

    def iter_log(self):
        """Rows (Phi before, Phi accepted, step size, halvings), one per accepted Newton iterate of the last step."""
        n = lib().ipco_iter_log(self.h, None, 0)
        out = np.zeros((max(n, 1), 4))
        lib().ipco_iter_log(self.h, _d(out), n)
        return out[:n]

    def inversion_bound(self, x, p):
        return lib().ipco_inversion_bound(self.h, _d(_f64(x)), _d(_f64(p)))

    @property
    def kappa(self):
        return lib().ipco_kappa(self.h)

    def contact_forces(self, x, tags, ntags):
        """[ntags, ntags, 3]: force on the vertices tagged a exerted by those tagged b, at x."""
        out = np.zeros((ntags, ntags, 3))
        _check(lib().ipco_contact_forces(self.h, _d(_f64(x)), _i(_i32(tags)), ntags, _d(out)))
        return out

    def hold_group(self, group, row):
        _check(lib().ipco_hold_group(self.h, int(group), int(row)))

    def set_gravity(self, g):
        _check(lib().ipco_set_gravity(self.h, None if g is None else _d(_f64(g))))

    def debug_ls_offset(self, delta):
        """Test-only planted fault: delta is added to every line-search trial energy."""
        lib().ipco_debug_ls_offset(self.h, float(delta))

    def friction_pairs(self):
        n = lib().ipco_friction_pairs(self.h, None, None, None, None, 0)
        v = np.zeros((max(n, 1), 4), np.int32)
        lam = np.zeros(max(n, 1))
        nrm = np.zeros((max(n, 1), 3))
        w = np.zeros((max(n, 1), 4))
        lib().ipco_friction_pairs(self.h, _i(v), _d(lam), _d(nrm), _d(w), n)
        return v[:n], lam[:n], nrm[:n], w[:n]


# --- element-level helpers -------------------------------------------------
def pt_classify(x12):
    d2 = C.c_double()
    t = lib().ipco_pt_classify(_d(_f64(x12).reshape(-1)), C.byref(d2))
    return t, d2.value


def ee_classify(x12):
    d2 = C.c_double()
    t = lib().ipco_ee_classify(_d(_f64(x12).reshape(-1)), C.byref(d2))
    return t, d2.value


def barrier_scalar(d, dhat):
    out = np.zeros(3)
    lib().ipco_barrier_scalar(d, dhat, _d(out))
    return out


def pair_barrier(kind, type_, x12, dhat, kappa, eps_x=0.0, project=False):
    e = C.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    lib().ipco_pair_barrier(kind, type_, _d(_f64(x12).reshape(-1)), dhat, kappa, eps_x, int(project), C.byref(e),
                            _d(g), _d(H))
    return e.value, g, H.reshape(12, 12)


def tet_elastic(X12, x12, E, nu, project=False):
    e = C.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    rc = lib().ipco_tet_elastic(_d(_f64(X12).reshape(-1)), _d(_f64(x12).reshape(-1)), E, nu, int(project),
                                C.byref(e), _d(g), _d(H))
    return rc, e.value, g, H.reshape(12, 12)


def psd_project(A):
    A = _f64(A).copy()
    n = A.shape[0]
    _check(lib().ipco_psd_project(n, _d(A)))
    return A


def accd(kind, x12, p12, s=0.1):
    return lib().ipco_accd(kind, _d(_f64(x12).reshape(-1)), _d(_f64(p12).reshape(-1)), s)


def friction_f0(y, eps):
    out = np.zeros(3)
    lib().ipco_friction_f0(y, eps, _d(out))
    return out


def friction_elem(x12, xn12, w4, n3, lam, mu, eps):
    e = C.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    lib().ipco_friction_elem(_d(_f64(x12).reshape(-1)), _d(_f64(xn12).reshape(-1)), _d(_f64(w4)), _d(_f64(n3)),
                             lam, mu, eps, C.byref(e), _d(g), _d(H))
    return e.value, g, H.reshape(12, 12)


def tet_first_root(x12, p12, tmax=1.25):
    """First t in (0, tmax] with det(Ds(x + t p)) <= 0 (inf if none), and the cubic's coefficients."""
    k = np.zeros(4)
    t = lib().ipco_tet_first_root(_d(_f64(x12).reshape(-1)), _d(_f64(p12).reshape(-1)), tmax, _d(k))
    return t, k
