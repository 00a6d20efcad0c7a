"""Python binding of libtrack.so (ctypes): argument marshalling only.

Every function keeps the name of the C entry point it calls (include/track.h).
Host arrays are numpy; device arrays may be torch tensors on the GPU (their
data pointer is passed with the on-device flag).  The library must have been
built (``paper_1711_07999_amd/_build.py``); importing this module on a
machine without it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrack.so")

TRACK_OK, TRACK_E_INVALID, TRACK_E_NOMEM, TRACK_E_DEVICE = 0, -1, -2, -3
TRACK_BLEND_DQ, TRACK_BLEND_LINEAR = 0, 1
TRACK_E_NOT_PD, TRACK_E_LOST, TRACK_E_BUDGET = -4, -5, -6
TRACK_GRAM_FP32, TRACK_GRAM_BF16X3, TRACK_GRAM_BF16X6 = 0, 1, 2

(TRACK_BUF_THETA, TRACK_BUF_PHI, TRACK_BUF_VERTS, TRACK_BUF_NORMALS, TRACK_BUF_DEPTH,
 TRACK_BUF_XYZ, TRACK_BUF_ASSOC, TRACK_BUF_COUNT, TRACK_BUF_DELTA, TRACK_BUF_GRAM,
 TRACK_BUF_STEP, TRACK_BUF_PHI_PREV, TRACK_BUF_VERTS_NEW) = range(13)
(TRACK_PASS_SKIN, TRACK_PASS_NORMALS, TRACK_PASS_ASSOCIATE, TRACK_PASS_NORMAL_EQ,
 TRACK_PASS_POSE_STEP, TRACK_PASS_SHAPE) = range(6)
(TRACK_K_SKIN, TRACK_K_NORMALS, TRACK_K_BUCKET, TRACK_K_ASSOC, TRACK_K_NORMAL_EQ,
 TRACK_K_SOLVE, TRACK_K_SHAPE) = range(7)
KERNEL_NAMES = ["skin", "normals", "bucket", "assoc", "normal_eq", "solve", "shape"]

EXPORTED = [
    "track_init", "track_frame", "track_frame_noalloc", "track_frame_xyz", "track_state",
    "track_joint_positions", "track_subdivide", "track_reset",
    "track_set_params", "track_destroy", "track_last_error", "track_dbg_set",
    "track_dbg_get", "track_dbg_run", "track_kernel_timing", "track_kernel_time", "track_kernel_bench",
    "track_server_create", "track_server_open", "track_server_submit", "track_server_step",
    "track_server_poll", "track_server_state", "track_server_close", "track_server_info",
    "track_server_destroy",
]


class TrackError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"track error {code}: {msg}")
        self.code = code


class track_model(ctypes.Structure):
    _fields_ = [
        ("n_joints", ctypes.c_int32), ("joint_parent", ctypes.c_void_p),
        ("joint_type", ctypes.c_void_p), ("joint_axis", ctypes.c_void_p),
        ("joint_offset", ctypes.c_void_p), ("n_links", ctypes.c_int32),
        ("link_joint", ctypes.c_void_p), ("n_verts", ctypes.c_int32),
        ("rest_xyz", ctypes.c_void_p), ("n_faces", ctypes.c_int32),
        ("faces", ctypes.c_void_p), ("max_infl", ctypes.c_int32),
        ("skin_link", ctypes.c_void_p), ("skin_w", ctypes.c_void_p),
        ("neighbors", ctypes.c_void_p), ("scale", ctypes.c_float), ("blend", ctypes.c_int32),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class track_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


def torch_allocator(device: int = 0, stream=None):
    """A track_allocator whose blocks come from PyTorch's caching allocator,
    so that torch counts and reuses a context's device memory.  The returned
    object counts its calls (``calls``) and must outlive the contexts made
    with it."""
    import torch

    st = torch.cuda.current_stream(device) if stream is None else stream
    calls = {"alloc": 0, "free": 0}

    def _alloc(nbytes, _user):
        calls["alloc"] += 1
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), device, st))
        except RuntimeError:
            return None

    def _free(ptr, _user):
        calls["free"] += 1
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))

    fns = (ALLOC_FN(_alloc), FREE_FN(_free))
    a = track_allocator(fns[0], fns[1], None)
    a.calls = calls
    a._fns = fns
    return a


class track_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class track_params(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_float), ("n_iters", ctypes.c_int32), ("do_pose", ctypes.c_void_p),
        ("do_shape", ctypes.c_void_p), ("lambda_k", ctypes.c_float), ("lambda_s", ctypes.c_float),
        ("lambda_phi", ctypes.c_float), ("lambda_nbr", ctypes.c_float), ("lambda_t", ctypes.c_float),
        ("lambda_w", ctypes.c_float), ("gram_mode", ctypes.c_int32),
        ("pose_solve_fp64", ctypes.c_int32), ("shape_solve_fp64", ctypes.c_int32),
        ("active", ctypes.c_void_p),
    ]


class track_frame_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_valid_px", ctypes.c_int32),
                ("n_assoc_px", ctypes.c_int32), ("n_obs_verts", ctypes.c_int32),
                ("energy_first", ctypes.c_float), ("energy_last", ctypes.c_float),
                ("step_norm_last", ctypes.c_float), ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class track_completion(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_int32), ("status", ctypes.c_int32), ("tag", ctypes.c_int64),
                ("stats", track_frame_stats)]


class track_server_stats(ctypes.Structure):
    _fields_ = [("resident", ctypes.c_int32), ("waiting", ctypes.c_int32),
                ("frames_in_progress", ctypes.c_int32), ("frames_pending", ctypes.c_int32),
                ("bytes_used", ctypes.c_int64), ("bytes_budget", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1711_07999_amd/_build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        sig = {
            "track_init": [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)],
            "track_frame": [vp, vp, i32],
            "track_frame_xyz": [vp, vp, i32],
            "track_frame_noalloc": [vp, vp, i32],
            "track_state": [vp, vp, vp, vp, vp],
            "track_joint_positions": [vp, vp],
            "track_subdivide": [vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp, vp, vp],
            "track_reset": [vp, vp, vp],
            "track_set_params": [vp, vp],
            "track_dbg_set": [vp, i32, vp, sz],
            "track_dbg_get": [vp, i32, vp, sz],
            "track_dbg_run": [vp, i32],
            "track_kernel_timing": [vp, i32, i32],
            "track_kernel_time": [vp, i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
            "track_kernel_bench": [vp, i32, vp, i32, ctypes.POINTER(ctypes.c_double)],
            "track_server_create": [vp, ctypes.c_int64, i32, vp, ctypes.POINTER(vp)],
            "track_server_open": [vp, vp, vp, vp, vp, ctypes.POINTER(i32)],
            "track_server_submit": [vp, i32, vp, i32, ctypes.c_int64],
            "track_server_step": [vp, ctypes.POINTER(i32)],
            "track_server_poll": [vp, vp, i32, ctypes.POINTER(i32)],
            "track_server_state": [vp, i32, vp, vp],
            "track_server_close": [vp, i32],
            "track_server_info": [vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.track_destroy.argtypes = [vp]
        L.track_destroy.restype = None
        L.track_server_destroy.argtypes = [vp]
        L.track_server_destroy.restype = None
        L.track_last_error.argtypes = []
        L.track_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def track_last_error() -> str:
    return lib().track_last_error().decode()


def _check(rc):
    if rc != TRACK_OK:
        raise TrackError(rc, track_last_error())
    return rc


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class _Keep:
    """Arrays whose memory a C struct points into."""

    def __init__(self):
        self.refs = []

    def __call__(self, a):
        self.refs.append(a)
        return _p(a)


def make_model(model: dict, keep: _Keep) -> track_model:
    nb = model.get("neighbors")
    m = track_model()
    m.n_joints = len(model["joint_parent"])
    m.joint_parent = keep(_c(model["joint_parent"], np.int32))
    m.joint_type = keep(_c(model["joint_type"], np.int32))
    m.joint_axis = keep(_c(model["joint_axis"], np.float32))
    m.joint_offset = keep(_c(model["joint_offset"], np.float32))
    m.n_links = len(model["link_joint"])
    m.link_joint = keep(_c(model["link_joint"], np.int32))
    m.n_verts = model["rest_xyz"].shape[0]
    m.rest_xyz = keep(_c(model["rest_xyz"], np.float32))
    m.n_faces = model["faces"].shape[0]
    m.faces = keep(_c(model["faces"], np.int32))
    m.max_infl = model["skin_link"].shape[1]
    m.skin_link = keep(_c(model["skin_link"], np.int32))
    m.skin_w = keep(_c(model["skin_w"], np.float32))
    m.neighbors = None if nb is None else keep(_c(nb, np.int32))
    m.scale = float(model.get("scale", 1.0))
    m.blend = int(model.get("blend", TRACK_BLEND_DQ))
    return m


def make_camera(cam: dict) -> track_camera:
    return track_camera(int(cam["width"]), int(cam["height"]), float(cam["fx"]), float(cam["fy"]),
                        float(cam["cx"]), float(cam["cy"]))


def make_params(prm: dict, keep: _Keep) -> track_params:
    n = int(prm["n_iters"])
    p = track_params()
    p.tau = float(prm["tau"])
    p.n_iters = n
    p.do_pose = keep(_c(prm["do_pose"], np.uint8))
    p.do_shape = keep(_c(prm["do_shape"], np.uint8))
    for k in ("lambda_k", "lambda_s", "lambda_phi", "lambda_nbr", "lambda_t", "lambda_w"):
        setattr(p, k, float(prm[k]))
    p.gram_mode = int(prm.get("gram_mode", 0))
    p.pose_solve_fp64 = int(prm.get("pose_solve_fp64", 0))
    p.shape_solve_fp64 = int(prm.get("shape_solve_fp64", 0))
    act = prm.get("active")
    p.active = None if act is None else keep(_c(act, np.uint8))
    return p


def _check_active(params: dict, P: int):
    act = params.get("active")
    if act is not None and np.asarray(act).shape != (P,):
        raise ValueError("params['active'] must hold one flag per joint")


def track_init(model: dict, camera: dict, params: dict, theta0, phi0=None, stream=None, allocator=None):
    """Returns an opaque context handle (ctypes.c_void_p).  ``allocator`` is a
    track_allocator (e.g. torch_allocator()) or None for the library's own."""
    keep = _Keep()
    m = make_model(model, keep)
    c = make_camera(camera)
    _check_active(params, m.n_joints)
    p = make_params(params, keep)
    th = _c(theta0, np.float64)
    if th.shape != (m.n_joints,):
        raise ValueError("theta0 must hold one value per joint")
    ph = None if phi0 is None else _c(phi0, np.float32)
    ctx = ctypes.c_void_p()
    st = None if stream is None else ctypes.c_void_p(int(stream))
    al = None if allocator is None else ctypes.byref(allocator)
    _check(lib().track_init(ctypes.byref(m), ctypes.byref(c), ctypes.byref(p), _p(th), _p(ph), st, al,
                            ctypes.byref(ctx)))
    return ctx


def _frame_ptr(x, dtype):
    """(pointer, on_device, keepalive) for a numpy array or a GPU torch tensor."""
    if hasattr(x, "is_cuda") and x.is_cuda:
        if not x.is_contiguous():
            raise ValueError("device frame must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), 1, x
    a = _c(x, dtype)
    return _p(a), 0, a


def track_frame(ctx, depth) -> int:
    ptr, dev, _k = _frame_ptr(depth, np.float32)
    rc = lib().track_frame(ctx, ptr, dev)
    return rc


def track_frame_noalloc(ctx, depth) -> int:
    ptr, dev, _k = _frame_ptr(depth, np.float32)
    return lib().track_frame_noalloc(ctx, ptr, dev)


def track_frame_xyz(ctx, xyz) -> int:
    ptr, dev, _k = _frame_ptr(xyz, np.float32)
    return lib().track_frame_xyz(ctx, ptr, dev)


def track_state(ctx, P: int, V: int, want_verts: bool = True):
    th = np.zeros(P, np.float64)
    ph = np.zeros((V, 3), np.float32)
    vv = np.zeros((V, 3), np.float32) if want_verts else None
    st = track_frame_stats()
    _check(lib().track_state(ctx, _p(th), _p(ph), _p(vv), ctypes.byref(st)))
    return th, ph, vv, st.as_dict()


def track_joint_positions(ctx, P: int):
    """[P, 3] float64 origins of the joint frames at the current pose."""
    out = np.zeros((P, 3))
    _check(lib().track_joint_positions(ctx, _p(out)))
    return out


class track_polymesh(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("n_faces", ctypes.c_int32),
                ("face_start", ctypes.c_void_p), ("face_verts", ctypes.c_void_p), ("max_infl", ctypes.c_int32),
                ("skin_link", ctypes.c_void_p), ("skin_w", ctypes.c_void_p)]


def track_subdivide(xyz, face_start, face_verts, skin_link, skin_w, levels: int = 2, max_infl_out: int = 4):
    """Catmull-Clark refinement of a polygon mesh with skin weights:
    returns (xyz [V',3] float32, tris [T',3] int32, skin_link [V',K] int32,
    skin_w [V',K] float32)."""
    x = _c(xyz, np.float32)
    fs = _c(face_start, np.int32)
    fv = _c(face_verts, np.int32)
    sl = _c(skin_link, np.int32)
    sw = _c(skin_w, np.float32)
    pm = track_polymesh(x.shape[0], _p(x), fs.shape[0] - 1, _p(fs), _p(fv), sl.shape[1], _p(sl), _p(sw))
    nv, nt = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().track_subdivide(ctypes.byref(pm), levels, max_infl_out, ctypes.byref(nv), ctypes.byref(nt),
                                 None, None, None, None))
    ox = np.zeros((nv.value, 3), np.float32)
    ot = np.zeros((nt.value, 3), np.int32)
    ol = np.zeros((nv.value, max_infl_out), np.int32)
    ow = np.zeros((nv.value, max_infl_out), np.float32)
    _check(lib().track_subdivide(ctypes.byref(pm), levels, max_infl_out, ctypes.byref(nv), ctypes.byref(nt),
                                 _p(ox), _p(ot), _p(ol), _p(ow)))
    return ox, ot, ol, ow


def track_reset(ctx, theta, phi=None):
    th = _c(theta, np.float64)
    ph = None if phi is None else _c(phi, np.float32)
    _check(lib().track_reset(ctx, _p(th), _p(ph)))


def track_set_params(ctx, params: dict):
    keep = _Keep()
    p = make_params(params, keep)
    _check(lib().track_set_params(ctx, ctypes.byref(p)))


def track_destroy(ctx):
    if ctx:
        lib().track_destroy(ctx)


def track_dbg_set(ctx, buf: int, arr):
    a = np.ascontiguousarray(arr)
    _check(lib().track_dbg_set(ctx, int(buf), _p(a), a.nbytes))


def track_dbg_get(ctx, buf: int, shape, dtype):
    a = np.zeros(shape, dtype)
    _check(lib().track_dbg_get(ctx, int(buf), _p(a), a.nbytes))
    return a


def track_dbg_run(ctx, pass_id: int) -> int:
    return lib().track_dbg_run(ctx, int(pass_id))


def track_kernel_timing(ctx, kernel: int, enable: bool):
    _check(lib().track_kernel_timing(ctx, int(kernel), int(bool(enable))))


def track_kernel_time(ctx, kernel: int):
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(lib().track_kernel_time(ctx, int(kernel), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def track_kernel_bench(ctx, kernel: int, depth, reps: int) -> float:
    """Mean ms of one launch of `kernel` over `reps` back-to-back launches;
    `depth` is a device tensor (or None for passes that read no image)."""
    ms = ctypes.c_double(0.0)
    ptr = None
    if depth is not None:
        if not (hasattr(depth, "is_cuda") and depth.is_cuda and depth.is_contiguous()):
            raise ValueError("depth must be a contiguous device tensor")
        ptr = ctypes.c_void_p(depth.data_ptr())
    _check(lib().track_kernel_bench(ctx, int(kernel), ptr, int(reps), ctypes.byref(ms)))
    return float(ms.value)


class Tracker:
    """Owns one context; convenience methods over the functions above."""

    def __init__(self, model: dict, camera: dict, params: dict, theta0, phi0=None, stream=None,
                 allocator=None):
        self.P = len(model["joint_parent"])
        self.V = model["rest_xyz"].shape[0]
        self.W, self.H = int(camera["width"]), int(camera["height"])
        self.allocator = allocator
        self.ctx = track_init(model, camera, params, theta0, phi0, stream, allocator)

    def frame(self, depth) -> int:
        return track_frame(self.ctx, depth)

    def frame_noalloc(self, depth) -> int:
        return track_frame_noalloc(self.ctx, depth)

    def frame_xyz(self, xyz) -> int:
        return track_frame_xyz(self.ctx, xyz)

    def state(self, want_verts=True):
        return track_state(self.ctx, self.P, self.V, want_verts)

    def joint_positions(self):
        return track_joint_positions(self.ctx, self.P)

    def reset(self, theta, phi=None):
        track_reset(self.ctx, theta, phi)

    def set_params(self, params):
        _check_active(params, self.P)
        track_set_params(self.ctx, params)

    def close(self):
        if self.ctx:
            track_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving -----------------------------------------------------------------
def track_server_create(params: dict, hbm_budget_bytes: int, max_streams: int, stream=None):
    keep = _Keep()
    p = make_params(dict(params, active=None), keep)
    sv = ctypes.c_void_p()
    st = None if stream is None else ctypes.c_void_p(int(stream))
    _check(lib().track_server_create(ctypes.byref(p), int(hbm_budget_bytes), int(max_streams), st,
                                     ctypes.byref(sv)))
    return sv


def track_server_open(sv, model: dict, camera: dict, theta0, phi0=None) -> int:
    keep = _Keep()
    m = make_model(model, keep)
    c = make_camera(camera)
    th = _c(theta0, np.float64)
    ph = None if phi0 is None else _c(phi0, np.float32)
    sid = ctypes.c_int32(-1)
    _check(lib().track_server_open(sv, ctypes.byref(m), ctypes.byref(c), _p(th), _p(ph), ctypes.byref(sid)))
    return int(sid.value)


def track_server_submit(sv, stream_id: int, depth, tag: int = 0):
    """depth: numpy (copied) or a GPU torch tensor (kept alive by the caller
    until its completion is polled)."""
    ptr, dev, _k = _frame_ptr(depth, np.float32)
    _check(lib().track_server_submit(sv, int(stream_id), ptr, dev, int(tag)))


def track_server_step(sv) -> int:
    n = ctypes.c_int32(0)
    _check(lib().track_server_step(sv, ctypes.byref(n)))
    return int(n.value)


def track_server_poll(sv, max_out: int = 1024):
    buf = (track_completion * max(1, max_out))()
    n = ctypes.c_int32(0)
    _check(lib().track_server_poll(sv, buf, int(max_out), ctypes.byref(n)))
    return [dict(buf[q].stats.as_dict(), stream=buf[q].stream, status=buf[q].status, tag=buf[q].tag)
            for q in range(n.value)]


def track_server_state(sv, stream_id: int, P: int, V: int):
    th = np.zeros(P, np.float64)
    ph = np.zeros((V, 3), np.float32)
    _check(lib().track_server_state(sv, int(stream_id), _p(th), _p(ph)))
    return th, ph


def track_server_close(sv, stream_id: int):
    _check(lib().track_server_close(sv, int(stream_id)))


def track_server_info(sv) -> dict:
    s = track_server_stats()
    _check(lib().track_server_info(sv, ctypes.byref(s)))
    return s.as_dict()


def track_server_destroy(sv):
    if sv:
        lib().track_server_destroy(sv)
