"""Python binding of the C-ABI in include/ipc.h (argument marshalling only).

Every computation runs in the HIP library ``libipc_mi355x.so``; this module
only converts numpy arrays to pointers.  Loading fails loudly when the
library has not been built: there is no other implementation behind it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipc_mi355x.so")

IPC_OK = 0
IPC_E_ARG = -1
IPC_E_INVERTED = -2
IPC_E_INTERSECTING = -3
IPC_E_NOMEM = -4
IPC_E_FAILED = -5
IPC_E_DEVICE = -6
IPC_FP64 = 0
IPC_MIXED = 1
IPC_TUNE_TAIL_TILES = 1
IPC_TUNE_FUSED_PCG = 2
IPC_TUNE_NARROW = 4
IPC_TUNE_LANES = 5
IPC_TUNE_ADMIT_FAULTS = 6
IPC_TUNE_ASYNC = 7
IPC_TUNE_WIDE_TILES = 8
IPC_TUNE_POLL_BLOCK = 9
IPC_TUNE_COARSE = 10
IPC_COARSE_BODIES = 4
IPC_FAIL_ADMIT = 6
FAIL_REASONS = {0: "none", 1: "maxit", 2: "nonfinite", 3: "line-search", 4: "dirichlet"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class ipc_scene_desc(C.Structure):
    _fields_ = [
        ("n_verts", C.c_int32), ("rest_pos", _dp), ("init_pos", _dp), ("init_vel", _dp),
        ("n_tets", C.c_int32), ("tets", _ip), ("E", _dp), ("nu", _dp), ("rho", _dp),
        ("n_tris", C.c_int32), ("tris", _ip), ("kin_group", _ip),
        ("n_groups", C.c_int32), ("n_motion_steps", C.c_int32), ("motion", _dp), ("gravity", _dp),
        ("dt", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double), ("mu", C.c_double),
        ("eps_v", C.c_double), ("newton_tol", C.c_double), ("newton_max_iter", C.c_int32),
        ("pcg_rel_tol", C.c_double), ("precision", C.c_int32),
        ("newton_rel_tol", C.c_double), ("friction_iters", C.c_int32), ("inversion_filter", C.c_int32),
        ("adaptive_kappa", C.c_int32),
    ]


class ipc_step_info(C.Structure):
    _fields_ = [
        ("steps_done", C.c_int32), ("status", C.c_int32), ("fail_reason", C.c_int32),
        ("newton_iters", C.c_int32), ("max_newton_iters", C.c_int32), ("ls_halvings", C.c_int32),
        ("pcg_iters", C.c_int64), ("n_active_last", C.c_int64), ("min_dist_last", C.c_double),
        ("energy_last", C.c_double), ("kappa_last", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "ipc_create_scene", "ipc_step", "ipc_step_batch", "ipc_get_state", "ipc_set_state", "ipc_destroy_scene",
    "ipc_last_error", "ipc_scene_sizes", "ipc_debug_candidates", "ipc_debug_active", "ipc_debug_begin_step",
    "ipc_debug_gradient", "ipc_debug_energy", "ipc_debug_hessian_apply", "ipc_debug_newton_dir", "ipc_debug_bodies",
    "ipc_debug_ccd_bound", "ipc_debug_classify", "ipc_debug_pair_barrier", "ipc_debug_tet_elastic",
    "ipc_debug_accd", "ipc_debug_inversion_bound", "ipc_debug_tet_first_root", "ipc_ccd_bound_pairs",
    "ipc_ccd_bound_pairs_noalloc", "ipc_grasp_metrics", "ipc_hold_group", "ipc_set_gravity", "ipc_contact_forces",
    "ipc_validate_grasp", "ipc_prof_enable", "ipc_prof_reset", "ipc_prof_read", "ipc_prof_pairs", "ipc_set_tuning", "ipc_get_tuning", "ipc_autotune",
    "ipc_server_create", "ipc_server_submit", "ipc_server_poll", "ipc_server_wait", "ipc_server_result",
    "ipc_server_release", "ipc_server_set_slots", "ipc_server_stats", "ipc_server_destroy",
]

IPC_REQ_QUEUED, IPC_REQ_RUNNING, IPC_REQ_DONE, IPC_REQ_FAILED = 0, 1, 2, 3
IPC_MAX_FINGERS = 8


class ipc_grasp_protocol(C.Structure):
    _fields_ = [
        ("vertex_tag", _ip), ("n_fingers", C.c_int32), ("finger_of_group", _ip), ("force_limit", C.c_double),
        ("max_close_steps", C.c_int32), ("settle_steps", C.c_int32), ("phase_steps", C.c_int32),
        ("gravity", C.c_double), ("com_factor", C.c_double),
    ]


class ipc_grasp_result(C.Structure):
    _fields_ = [
        ("stable", C.c_int32), ("in_contact", C.c_int32), ("failed", C.c_int32), ("fail_reason", C.c_int32),
        ("steps_run", C.c_int32), ("halt_step", C.c_int32 * IPC_MAX_FINGERS),
        ("finger_force", C.c_double * IPC_MAX_FINGERS), ("com_shift", C.c_double * 6), ("com_drift", C.c_double * 6),
    ]


class ipc_request_info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("steps_done", C.c_int32), ("n_steps", C.c_int32), ("fail_reason", C.c_int32),
        ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
        ("newton_iters", C.c_int64), ("pcg_iters", C.c_int64), ("bytes", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2503_05020_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.ipc_create_scene.argtypes = [C.POINTER(ipc_scene_desc), C.POINTER(vp)]
    L.ipc_step.argtypes = [vp, C.c_int32, C.POINTER(ipc_step_info)]
    L.ipc_step_batch.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.POINTER(ipc_step_info)]
    L.ipc_get_state.argtypes = [vp, _dp, _dp, _dp, _dp]
    L.ipc_set_state.argtypes = [vp, _dp, _dp, C.c_int32]
    L.ipc_destroy_scene.argtypes = [vp]
    L.ipc_destroy_scene.restype = None
    L.ipc_last_error.restype = C.c_char_p
    L.ipc_scene_sizes.argtypes = [vp, C.POINTER(C.c_int64)]
    L.ipc_debug_candidates.argtypes = [vp, _dp, _dp, _ip, C.c_int64]
    L.ipc_debug_candidates.restype = C.c_int64
    L.ipc_debug_active.argtypes = [vp, _dp, _ip, _dp, C.c_int64]
    L.ipc_debug_active.restype = C.c_int64
    L.ipc_debug_begin_step.argtypes = [vp, _dp]
    L.ipc_debug_gradient.argtypes = [vp, _dp, _dp]
    L.ipc_debug_energy.argtypes = [vp, _dp]
    L.ipc_debug_energy.restype = C.c_double
    L.ipc_debug_hessian_apply.argtypes = [vp, _dp, _dp, _dp]
    L.ipc_debug_newton_dir.argtypes = [vp, _dp, _dp, C.POINTER(C.c_int64)]
    L.ipc_debug_bodies.argtypes = [vp, _ip, _dp]
    L.ipc_debug_ccd_bound.argtypes = [vp, _dp, _dp]
    L.ipc_debug_ccd_bound.restype = C.c_double
    L.ipc_debug_classify.argtypes = [C.c_int32, C.c_int64, _dp, _ip, _dp]
    L.ipc_debug_pair_barrier.argtypes = [C.c_int32, C.c_int32, _dp, C.c_double, C.c_double, C.c_double, C.c_int32,
                                         _dp, _dp, _dp]
    L.ipc_debug_tet_elastic.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_int32, _dp, _dp, _dp]
    L.ipc_debug_accd.argtypes = [C.c_int32, C.c_int64, _dp, _dp, C.c_double, _dp]
    L.ipc_debug_accd.restype = C.c_int64
    L.ipc_ccd_bound_pairs.argtypes = [C.c_int32, C.c_int64, _dp, _dp, C.c_double, _dp]
    L.ipc_grasp_metrics.argtypes = [vp, C.c_int32, _ip, C.c_int32, _ip, C.c_int32, _ip, _dp, _dp, _dp]
    L.ipc_hold_group.argtypes = [vp, C.c_int32, C.c_int32]
    L.ipc_set_gravity.argtypes = [vp, _dp]
    L.ipc_contact_forces.argtypes = [vp, _ip, C.c_int32, _dp]
    L.ipc_validate_grasp.argtypes = [vp, C.POINTER(ipc_grasp_protocol), C.POINTER(ipc_grasp_result)]
    L.ipc_ccd_bound_pairs_noalloc.argtypes = [C.c_int32, C.c_int64, vp, vp, C.c_double, vp, vp]
    L.ipc_debug_inversion_bound.argtypes = [vp, _dp, _dp]
    L.ipc_debug_inversion_bound.restype = C.c_double
    L.ipc_debug_tet_first_root.argtypes = [C.c_int64, _dp, _dp, C.c_double, _dp, _dp]
    L.ipc_debug_tet_first_root.restype = C.c_int64
    L.ipc_prof_enable.argtypes = [C.c_int32]
    L.ipc_prof_read.argtypes = [_dp]
    L.ipc_prof_pairs.argtypes = [_dp]
    L.ipc_set_tuning.argtypes = [C.c_int32, C.c_int64]
    L.ipc_get_tuning.argtypes = [C.c_int32, C.POINTER(C.c_int64)]
    L.ipc_autotune.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_char_p, C.POINTER(C.c_int64)]
    L.ipc_server_create.argtypes = [C.c_int64, C.c_int32, C.POINTER(vp)]
    L.ipc_server_submit.argtypes = [vp, C.POINTER(ipc_scene_desc), C.c_int32, C.POINTER(C.c_int64)]
    L.ipc_server_poll.argtypes = [vp, C.c_int64, C.POINTER(ipc_request_info)]
    L.ipc_server_wait.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(ipc_request_info)]
    L.ipc_server_result.argtypes = [vp, C.c_int64, _dp, _dp]
    L.ipc_server_release.argtypes = [vp, C.c_int64]
    L.ipc_server_set_slots.argtypes = [vp, C.c_int32]
    L.ipc_server_stats.argtypes = [vp, _dp]
    L.ipc_server_destroy.argtypes = [vp]
    L.ipc_server_destroy.restype = None
    _lib = L
    return L


class IPCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ipc error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise IPCError(rc, lib().ipc_last_error().decode())
    return rc


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _i(a):
    return None if a is None else a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def ipc_last_error() -> str:
    return lib().ipc_last_error().decode()


def make_desc(sc: dict, precision: int = IPC_FP64, pcg_rel_tol: float = 1e-4, **overrides):
    """Build an ipc_scene_desc from a scene dict; returns (desc, keep-alive arrays)."""
    p = dict(sc)
    p.update(overrides)
    keep = dict(
        rest=_f64(p["rest_pos"]).reshape(-1),
        init=_f64(p.get("init_pos", p["rest_pos"])).reshape(-1),
        vel=_f64(p.get("init_vel", np.zeros_like(p["rest_pos"]))).reshape(-1),
        tets=np.ascontiguousarray(p["tets"], np.int32).reshape(-1),
        E=_f64(p["E"]), nu=_f64(p["nu"]), rho=_f64(p["rho"]),
        tris=np.ascontiguousarray(p["tris"], np.int32).reshape(-1),
        kin=np.ascontiguousarray(p["kin_group"], np.int32),
        motion=_f64(p["motion"]).reshape(-1), gravity=_f64(p["gravity"]).reshape(-1),
    )
    motion = np.asarray(p["motion"])
    if motion.ndim != 3 or motion.shape[2] != 12 or np.asarray(p["gravity"]).reshape(-1, 3).shape[0] != motion.shape[0]:
        raise ValueError("motion must be [steps][groups][12] with one gravity row per step")
    d = ipc_scene_desc(
        len(keep["kin"]), _d(keep["rest"]), _d(keep["init"]), _d(keep["vel"]),
        len(keep["E"]), _i(keep["tets"]), _d(keep["E"]), _d(keep["nu"]), _d(keep["rho"]),
        len(keep["tris"]) // 3, _i(keep["tris"]), _i(keep["kin"]),
        motion.shape[1], motion.shape[0], _d(keep["motion"]), _d(keep["gravity"]),
        p["dt"], p["dhat"], p["kappa"], p["mu"], p["eps_v"], p["newton_tol"], int(p["newton_max_iter"]),
        pcg_rel_tol, precision, float(p.get("newton_rel_tol", 0.0)), int(p.get("friction_iters", 1)),
        int(p.get("inversion_filter", 0)), int(p.get("adaptive_kappa", 0)))
    return d, keep


def ipc_create_scene(sc: dict, precision: int = IPC_FP64, pcg_rel_tol: float = 1e-4, **overrides) -> "Scene":
    d, keep = make_desc(sc, precision, pcg_rel_tol, **overrides)
    h = C.c_void_p()
    _check(lib().ipc_create_scene(C.byref(d), C.byref(h)))
    return Scene(h, len(keep["kin"]), len(keep["E"]))


def ipc_step(scene: "Scene", n_steps: int = 1):
    info = ipc_step_info()
    rc = lib().ipc_step(scene.h, n_steps, C.byref(info))
    if rc < 0 and rc != IPC_E_FAILED:
        _check(rc)
    return rc, info.as_dict()


def ipc_step_batch(scenes, n_steps: int = 1):
    arr = (C.c_void_p * len(scenes))(*[s.h.value for s in scenes])
    infos = (ipc_step_info * max(1, len(scenes)))()
    rc = lib().ipc_step_batch(arr, len(scenes), n_steps, infos)
    if rc < 0 and rc != IPC_E_FAILED:
        _check(rc)
    return rc, [infos[i].as_dict() for i in range(len(scenes))]


def ipc_get_state(scene: "Scene", stress: bool = False):
    pos = np.zeros((scene.nv, 3))
    vel = np.zeros((scene.nv, 3))
    cau = np.zeros((scene.nt, 6)) if stress else None
    vm = np.zeros(scene.nt) if stress else None
    _check(lib().ipc_get_state(scene.h, _d(pos), _d(vel), _d(cau), _d(vm)))
    return (pos, vel, cau, vm) if stress else (pos, vel)


def ipc_set_state(scene: "Scene", pos, vel=None, step: int = 0):
    v = None if vel is None else _f64(vel)
    _check(lib().ipc_set_state(scene.h, _d(_f64(pos)), _d(v), step))


def ipc_destroy_scene(scene: "Scene"):
    if scene.h is not None and _lib is not None:
        _lib.ipc_destroy_scene(scene.h)
        scene.h = None


def ipc_scene_sizes(scene: "Scene"):
    out = (C.c_int64 * 7)()
    _check(lib().ipc_scene_sizes(scene.h, out))
    return list(out)


class Scene:
    """Handle of a scene living in device memory."""

    def __init__(self, h, nv, nt):
        self.h, self.nv, self.nt = h, nv, nt

    def __del__(self):
        try:
            ipc_destroy_scene(self)
        except Exception:
            pass

    # convenience wrappers
    def step(self, n=1):
        return ipc_step(self, n)

    def state(self, stress=False):
        return ipc_get_state(self, stress)


# --- measurement ----------------------------------------------------------------
def ipc_prof_enable(on=1):
    _check(lib().ipc_prof_enable(int(on)))


def ipc_prof_reset():
    _check(lib().ipc_prof_reset())


def ipc_prof_read():
    out = np.zeros(12)
    _check(lib().ipc_prof_read(_d(out)))
    return {"spmv_ms": float(out[0]), "spmv_launches": int(out[1]), "spmv_bytes": float(out[2]),
            "big_ms": float(out[3]), "big_launches": int(out[4]), "big_bytes": float(out[5]),
            "iter_ms": float(out[6]), "iters": int(out[7]), "iter_bytes": float(out[8]),
            "asm_ms": float(out[9]), "asm_passes": int(out[10]), "asm_bytes": float(out[11])}


def ipc_prof_pairs():
    """Contact work since the last reset: candidates classified, barrier and friction elements evaluated."""
    out = np.zeros(3)
    _check(lib().ipc_prof_pairs(_d(out)))
    return {"candidates": int(out[0]), "barrier_elems": int(out[1]), "friction_elems": int(out[2])}


def ipc_set_tuning(key: int, value: int):
    _check(lib().ipc_set_tuning(key, int(value)))


def ipc_get_tuning(key: int) -> int:
    out = C.c_int64()
    _check(lib().ipc_get_tuning(key, C.byref(out)))
    return int(out.value)


def ipc_autotune(scenes, steps: int = 2, cache_path=None):
    """Per-workload choice of IPC_TUNE_WIDE_TILES and IPC_TUNE_POLL_BLOCK (applied to the device);
    returns (wide_tiles, poll_block, from_cache)."""
    arr = (C.c_void_p * max(1, len(scenes)))(*[s.h.value for s in scenes])
    out = (C.c_int64 * 3)()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().ipc_autotune(arr, len(scenes), int(steps), path, out))
    return int(out[0]), int(out[1]), bool(out[2])


# --- serving -----------------------------------------------------------------
class Server:
    """Handle of a serving loop on the current device (see ipc_server_* in ipc.h)."""

    def __init__(self, h):
        self.h = h
        self.nv = {}


def ipc_server_create(budget_bytes: int, max_slots: int) -> Server:
    h = C.c_void_p()
    _check(lib().ipc_server_create(int(budget_bytes), int(max_slots), C.byref(h)))
    return Server(h)


def ipc_server_submit(srv: Server, sc: dict, n_steps: int, precision: int = IPC_FP64, pcg_rel_tol: float = 1e-4,
                      **overrides) -> int:
    d, keep = make_desc(sc, precision, pcg_rel_tol, **overrides)
    rid = C.c_int64()
    _check(lib().ipc_server_submit(srv.h, C.byref(d), int(n_steps), C.byref(rid)))
    srv.nv[rid.value] = len(keep["kin"])
    return int(rid.value)


def ipc_server_poll(srv: Server, rid: int) -> dict:
    info = ipc_request_info()
    _check(lib().ipc_server_poll(srv.h, int(rid), C.byref(info)))
    return info.as_dict()


def ipc_server_wait(srv: Server, rid: int, timeout_s: float = 1e6) -> dict:
    info = ipc_request_info()
    _check(lib().ipc_server_wait(srv.h, int(rid), float(timeout_s), C.byref(info)))
    return info.as_dict()


def ipc_server_result(srv: Server, rid: int):
    n = srv.nv[int(rid)]
    pos = np.zeros((n, 3))
    vel = np.zeros((n, 3))
    _check(lib().ipc_server_result(srv.h, int(rid), _d(pos), _d(vel)))
    return pos, vel


def ipc_server_release(srv: Server, rid: int):
    _check(lib().ipc_server_release(srv.h, int(rid)))
    srv.nv.pop(int(rid), None)


def ipc_server_set_slots(srv: Server, max_slots: int):
    _check(lib().ipc_server_set_slots(srv.h, int(max_slots)))


def ipc_server_stats(srv: Server) -> dict:
    out = np.zeros(9)
    _check(lib().ipc_server_stats(srv.h, _d(out)))
    keys = ["finished", "failed", "converged_steps", "ticks", "running", "queued", "bytes_in_use", "seconds",
            "slot_cap"]
    return dict(zip(keys, out.tolist()))


def ipc_server_destroy(srv: Server):
    if srv.h is not None and _lib is not None:
        _lib.ipc_server_destroy(srv.h)
        srv.h = None


# --- inspection entry points -------------------------------------------------
def ipc_debug_candidates(scene, x, p=None):
    x = _f64(x)
    p = None if p is None else _f64(p)
    n = _check(lib().ipc_debug_candidates(scene.h, _d(x), _d(p), None, 0))
    out = np.zeros((max(n, 1), 5), np.int32)
    _check(lib().ipc_debug_candidates(scene.h, _d(x), _d(p), _i(out), n))
    return out[:n]


def ipc_debug_active(scene, x):
    x = _f64(x)
    n = _check(lib().ipc_debug_active(scene.h, _d(x), None, None, 0))
    out = np.zeros((max(n, 1), 6), np.int32)
    d2 = np.zeros(max(n, 1))
    _check(lib().ipc_debug_active(scene.h, _d(x), _i(out), _d(d2), n))
    return out[:n], d2[:n]


def ipc_debug_begin_step(scene):
    x0 = np.zeros((scene.nv, 3))
    _check(lib().ipc_debug_begin_step(scene.h, _d(x0)))
    return x0


def ipc_debug_gradient(scene, x):
    g = np.zeros((scene.nv, 3))
    _check(lib().ipc_debug_gradient(scene.h, _d(_f64(x)), _d(g)))
    return g


def ipc_debug_energy(scene, x):
    return lib().ipc_debug_energy(scene.h, _d(_f64(x)))


def ipc_debug_hessian_apply(scene, x, v):
    y = np.zeros((scene.nv, 3))
    _check(lib().ipc_debug_hessian_apply(scene.h, _d(_f64(x)), _d(_f64(v)), _d(y)))
    return y


def ipc_debug_newton_dir(scene, x):
    p = np.zeros((scene.nv, 3))
    it = C.c_int64()
    _check(lib().ipc_debug_newton_dir(scene.h, _d(_f64(x)), _d(p), C.byref(it)))
    return p, it.value


def ipc_debug_bodies(scene):
    """Per-vertex body of the two-level PCG's coarse space and each body's (x, y, z, size)."""
    vbody = np.zeros(scene.nv, np.int32)
    frame = np.zeros((IPC_COARSE_BODIES, 4))
    n = lib().ipc_debug_bodies(scene.h, _i(vbody), _d(frame))
    _check(n)
    return vbody, frame[:n]


def ipc_debug_ccd_bound(scene, x, p):
    return lib().ipc_debug_ccd_bound(scene.h, _d(_f64(x)), _d(_f64(p)))


def ipc_ccd_bound_pairs(kind, x12, p12, s=0.1):
    """min(1, min over the pairs of the additive-CCD time of impact) for pairs of one kind."""
    x12 = _f64(x12).reshape(-1, 12)
    p12 = _f64(p12).reshape(-1, 12)
    a = C.c_double()
    _check(lib().ipc_ccd_bound_pairs(kind, len(x12), _d(x12), _d(p12), s, C.byref(a)))
    return a.value


def ipc_ccd_bound_pairs_noalloc(kind, n, x12_dev, p12_dev, alpha_dev, s=0.1, stream=None):
    """Allocation-free variant: device addresses (ints) of x12 [n*12], p12 [n*12] and alpha [1] FP64
    buffers; queued on `stream` (a hipStream_t handle as an int, None = null stream), not waited for."""
    _check(lib().ipc_ccd_bound_pairs_noalloc(kind, n, x12_dev, p12_dev, s, alpha_dev, stream))


def ipc_grasp_metrics(scene, obj_tris, hand_tris, sample_tri, sample_uv, want_sdf=False):
    """D1, D2 (Sec. IV-C Eq. (2)-(3)) at the scene's current positions; with want_sdf also d_o at every sample."""
    ot = np.ascontiguousarray(obj_tris, np.int32).reshape(-1, 3)
    ht = np.ascontiguousarray(hand_tris, np.int32).reshape(-1, 3)
    st = np.ascontiguousarray(sample_tri, np.int32).reshape(-1)
    uv = _f64(sample_uv).reshape(-1, 2)
    D = np.zeros(2)
    sdf = np.zeros(len(st)) if want_sdf else None
    _check(lib().ipc_grasp_metrics(scene.h, len(ot), _i(ot), len(ht), _i(ht), len(st), _i(st), _d(uv), _d(D),
                                   _d(sdf)))
    return (D[0], D[1], sdf) if want_sdf else (D[0], D[1])


def ipc_hold_group(scene, group, row):
    _check(lib().ipc_hold_group(scene.h, int(group), int(row)))


def ipc_set_gravity(scene, g):
    _check(lib().ipc_set_gravity(scene.h, None if g is None else _d(_f64(g).reshape(3))))


def ipc_contact_forces(scene, tags, ntags):
    """[ntags, ntags, 3]: force on the vertices tagged a exerted by those tagged b."""
    t = np.ascontiguousarray(tags, np.int32)
    out = np.zeros((ntags, ntags, 3))
    _check(lib().ipc_contact_forces(scene.h, _i(t), int(ntags), _d(out)))
    return out


def ipc_validate_grasp(scene, vertex_tag, n_fingers, finger_of_group, force_limit=50.0, max_close_steps=60,
                       settle_steps=10, phase_steps=10, gravity=9.8, com_factor=10.0):
    vt = np.ascontiguousarray(vertex_tag, np.int32)
    fg = np.ascontiguousarray(finger_of_group, np.int32)
    p = ipc_grasp_protocol(_i(vt), int(n_fingers), _i(fg), float(force_limit), int(max_close_steps),
                           int(settle_steps), int(phase_steps), float(gravity), float(com_factor))
    r = ipc_grasp_result()
    _check(lib().ipc_validate_grasp(scene.h, C.byref(p), C.byref(r)))
    return {"stable": r.stable, "in_contact": r.in_contact, "failed": r.failed, "fail_reason": r.fail_reason,
            "steps_run": r.steps_run, "halt_step": list(r.halt_step)[:n_fingers],
            "finger_force": list(r.finger_force)[:n_fingers], "com_shift": list(r.com_shift),
            "com_drift": list(r.com_drift)}


def ipc_debug_inversion_bound(scene, x, p):
    return lib().ipc_debug_inversion_bound(scene.h, _d(_f64(x)), _d(_f64(p)))


def ipc_debug_tet_first_root(x12, p12, tmax=1.25):
    """Per tet: first root of det(Ds(x + t p)) in (0, tmax] and the cubic's coefficients [n, 4]."""
    x12 = _f64(x12).reshape(-1, 12)
    p12 = _f64(p12).reshape(-1, 12)
    n = len(x12)
    t = np.zeros(n)
    k = np.zeros((n, 4))
    _check(lib().ipc_debug_tet_first_root(n, _d(x12), _d(p12), tmax, _d(t), _d(k)))
    return t, k


def ipc_debug_classify(kind, x12):
    x12 = _f64(x12).reshape(-1, 12)
    n = len(x12)
    t = np.zeros(n, np.int32)
    d2 = np.zeros(n)
    _check(lib().ipc_debug_classify(kind, n, _d(x12), _i(t), _d(d2)))
    return t, d2


def ipc_debug_pair_barrier(kind, type_, x12, dhat, kappa, eps_x=0.0, project=True):
    e = C.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    _check(lib().ipc_debug_pair_barrier(kind, type_, _d(_f64(x12).reshape(-1)), dhat, kappa, eps_x, int(project),
                                        C.byref(e), _d(g), _d(H)))
    return e.value, g, H.reshape(12, 12)


def ipc_debug_tet_elastic(X12, x12, E, nu):
    e = C.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    rc = lib().ipc_debug_tet_elastic(_d(_f64(X12).reshape(-1)), _d(_f64(x12).reshape(-1)), E, nu, 1, C.byref(e),
                                     _d(g), _d(H))
    return rc, e.value, g, H.reshape(12, 12)


def ipc_debug_accd(kind, x12, p12, s=0.1):
    x12 = _f64(x12).reshape(-1, 12)
    p12 = _f64(p12).reshape(-1, 12)
    n = len(x12)
    t = np.zeros(n)
    _check(lib().ipc_debug_accd(kind, n, _d(x12), _d(p12), s, _d(t)))
    return t
