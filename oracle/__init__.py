"""CPU oracle of the per-frame tracking step (ctypes wrapper of liboracle.so).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never does, and
this package imports nothing from it.

Each function mirrors one step of the paper's method (see oracle.hpp for the
section and equation each follows); all floating point is float64 except the
association decisions, which are taken in float32 with the operation order
stated in oracle.hpp.  track_frame(..., fp32=True) runs a float32
instantiation of the same source, for the CPU timing baseline only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([
            "g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
            "-fopenmp", "-fPIC", "-shared", os.path.join(_HERE, "capi.cpp"),
            os.path.join(_HERE, "capi32.cpp"), "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Model(ctypes.Structure):
    _fields_ = [
        ("n_joints", ctypes.c_int32), ("joint_parent", ctypes.c_void_p),
        ("joint_type", ctypes.c_void_p), ("joint_axis", ctypes.c_void_p),
        ("joint_offset", ctypes.c_void_p), ("n_links", ctypes.c_int32),
        ("link_joint", ctypes.c_void_p), ("n_verts", ctypes.c_int32),
        ("rest_xyz", ctypes.c_void_p), ("n_faces", ctypes.c_int32),
        ("faces", ctypes.c_void_p), ("max_infl", ctypes.c_int32),
        ("skin_link", ctypes.c_void_p), ("skin_w", ctypes.c_void_p),
        ("neighbors", ctypes.c_void_p), ("blend", ctypes.c_int32),
    ]


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class _Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_float), ("n_iters", ctypes.c_int32),
                ("do_pose", ctypes.c_void_p), ("do_shape", ctypes.c_void_p),
                ("active", ctypes.c_void_p), ("lambda_k", ctypes.c_double),
                ("lambda_s", ctypes.c_double), ("lambda_phi", ctypes.c_double),
                ("lambda_nbr", ctypes.c_double), ("lambda_t", ctypes.c_double),
                ("lambda_w", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        _lib = ctypes.CDLL(LIB_PATH)
        for name in ("orc_fk", "orc_skin", "orc_normals", "orc_skin_dual", "orc_transform",
                     "orc_associate", "orc_average", "orc_pose_system",
                     "orc_prior_weights", "orc_lm_solve", "orc_shape_step", "orc_shape_step_literal",
                     "orc_track_frame", "orc32_track_frame", "orc_set_threads"):
            getattr(_lib, name).restype = ctypes.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Model:
    """Holds contiguous copies of a model dictionary and its C view."""

    def __init__(self, model: dict):
        self.arrays = {
            "joint_parent": _c(model["joint_parent"], np.int32),
            "joint_type": _c(model["joint_type"], np.int32),
            "joint_axis": _c(model["joint_axis"], np.float32),
            "joint_offset": _c(model["joint_offset"], np.float32),
            "link_joint": _c(model["link_joint"], np.int32),
            "rest_xyz": _c(model["rest_xyz"], np.float32),
            "faces": _c(model["faces"], np.int32),
            "skin_link": _c(model["skin_link"], np.int32),
            "skin_w": _c(model["skin_w"], np.float32),
        }
        nb = model.get("neighbors")
        self.arrays["neighbors"] = None if nb is None else _c(nb, np.int32)
        a = self.arrays
        self.P = a["joint_parent"].shape[0]
        self.L = a["link_joint"].shape[0]
        self.V = a["rest_xyz"].shape[0]
        self.F = a["faces"].shape[0]
        self.K = a["skin_link"].shape[1]
        self.c = _Model(self.P, _p(a["joint_parent"]), _p(a["joint_type"]),
                        _p(a["joint_axis"]), _p(a["joint_offset"]), self.L,
                        _p(a["link_joint"]), self.V, _p(a["rest_xyz"]), self.F,
                        _p(a["faces"]), self.K, _p(a["skin_link"]),
                        _p(a["skin_w"]), _p(a["neighbors"]), int(model.get("blend", 0)))


def _model(m):
    return m if isinstance(m, Model) else Model(m)


def _cam(c: dict):
    return _Camera(int(c["width"]), int(c["height"]), float(c["fx"]), float(c["fy"]),
                   float(c["cx"]), float(c["cy"]))


def set_threads(n: int) -> int:
    return lib().orc_set_threads(int(n))


def fk(model, theta):
    """(H_0j [P,8], H_lDelta [L,8]) as (r.w r.x r.y r.z d.w d.x d.y d.z)."""
    m = _model(model)
    th = _c(theta, np.float64)
    Hj = np.zeros((m.P, 8))
    dH = np.zeros((m.L, 8))
    lib().orc_fk(ctypes.byref(m.c), _p(th), _p(Hj), _p(dH))
    return Hj, dH


def skin(model, theta, phi=None):
    """Skinned vertices v [V,3] and unit vertex normals n [V,3] (float64)."""
    m = _model(model)
    th = _c(theta, np.float64)
    ph = np.zeros((m.V, 3)) if phi is None else _c(phi, np.float64)
    v = np.zeros((m.V, 3))
    n = np.zeros((m.V, 3))
    lib().orc_skin(ctypes.byref(m.c), _p(th), _p(ph), _p(v), _p(n))
    return v, n


def normals(model, v):
    """Unit vertex normals of the given vertex positions (float64)."""
    m = _model(model)
    vv = _c(v, np.float64)
    n = np.zeros((m.V, 3))
    lib().orc_normals(ctypes.byref(m.c), _p(vv), _p(n))
    return n


def skin_dual(model, theta, dtheta=None, phi=None, dphi=None):
    """Skinned vertices and their forward-mode derivative along (dtheta, dphi)."""
    m = _model(model)
    th = _c(theta, np.float64)
    dth = None if dtheta is None else _c(dtheta, np.float64)
    ph = np.zeros((m.V, 3)) if phi is None else _c(phi, np.float64)
    dph = None if dphi is None else _c(dphi, np.float64)
    v = np.zeros((m.V, 3))
    dv = np.zeros((m.V, 3))
    lib().orc_skin_dual(ctypes.byref(m.c), _p(th), _p(dth), _p(ph), _p(dph), _p(v), _p(dv))
    return v, dv


def transform(H8, x):
    """T(H, x) and dT/dH [3,8] for one (blended) dual quaternion."""
    H = _c(H8, np.float64)
    xx = _c(x, np.float64)
    T = np.zeros(3)
    J = np.zeros((3, 8))
    lib().orc_transform(_p(H), _p(xx), _p(T), _p(J))
    return T, J


def associate(cam, tau, v32, depth=None, xyz=None, brute=False):
    """a(k) per pixel (int32 [H*W]); v32 is float32 [V,3]."""
    v = _c(v32, np.float32)
    a = np.empty(int(cam["width"]) * int(cam["height"]), np.int32)
    d = None if depth is None else _c(depth, np.float32)
    x = None if xyz is None else _c(xyz, np.float32)
    c = _cam(cam)
    lib().orc_associate(ctypes.byref(c), ctypes.c_float(tau), _p(v), v.shape[0], _p(d), _p(x),
                        int(bool(brute)), _p(a))
    return a


def average(cam, a, v, depth=None, xyz=None):
    """(c_i int32 [V], delta_i float64 [V,3]) from an association."""
    vv = _c(v, np.float64)
    V = vv.shape[0]
    cnt = np.zeros(V, np.int32)
    delta = np.zeros((V, 3))
    d = None if depth is None else _c(depth, np.float32)
    x = None if xyz is None else _c(xyz, np.float32)
    aa = _c(a, np.int32)
    c = _cam(cam)
    lib().orc_average(ctypes.byref(c), _p(d), _p(x), _p(aa), _p(vv), V, _p(cnt), _p(delta))
    return cnt, delta


def pose_system(model, theta, phi, n, delta, cnt, lambda_s=0.0):
    """dict(J [V,P], r [V], A [P,P], b [P], rr)."""
    m = _model(model)
    th = _c(theta, np.float64)
    ph = _c(phi, np.float64)
    nn = _c(n, np.float64)
    de = _c(delta, np.float64)
    cc = _c(cnt, np.int32)
    J = np.zeros((m.V, m.P))
    r = np.zeros(m.V)
    A = np.zeros((m.P, m.P))
    b = np.zeros(m.P)
    rr = ctypes.c_double(0.0)
    lib().orc_pose_system(ctypes.byref(m.c), _p(th), _p(ph), _p(nn), _p(de), _p(cc),
                          ctypes.c_double(lambda_s), _p(J), _p(r), _p(A), _p(b), ctypes.byref(rr))
    return dict(J=J, r=r, A=A, b=b, rr=rr.value)


def prior_weights(model):
    m = _model(model)
    out = np.zeros(m.P)
    lib().orc_prior_weights(ctypes.byref(m.c), _p(out))
    return out


def lm_solve(A, b, lambda_k, active=None):
    """Damped step x; raises on a failed factorisation."""
    AA = _c(A, np.float64)
    bb = _c(b, np.float64)
    P = bb.shape[0]
    x = np.zeros(P)
    act = None if active is None else _c(active, np.uint8)
    rc = lib().orc_lm_solve(P, _p(AA), _p(bb), ctypes.c_double(lambda_k), _p(act), _p(x))
    if rc != 0:
        raise np.linalg.LinAlgError(f"cholesky failed ({rc})")
    return x


def shape_step(model, theta, phi, phi_prev, n, delta, cnt, lambda_phi, lambda_nbr,
               lambda_t, lambda_w):
    m = _model(model)
    out = np.zeros((m.V, 3))
    args = [_c(theta, np.float64), _c(phi, np.float64), _c(phi_prev, np.float64),
            _c(n, np.float64), _c(delta, np.float64), _c(cnt, np.int32)]
    lib().orc_shape_step(ctypes.byref(m.c), *[_p(a) for a in args], ctypes.c_double(lambda_phi),
                         ctypes.c_double(lambda_nbr), ctypes.c_double(lambda_t),
                         ctypes.c_double(lambda_w), _p(out))
    return out


def shape_step_literal(model, theta, phi, n, delta, cnt, lambda_phi, lambda_nbr, lambda_w):
    """Eq. (9) as printed (one scalar residual per vertex with the
    regularisers inside it, rank-one normal matrix plus its own diagonal):
    kept to demonstrate why the least-squares reading is used."""
    m = _model(model)
    out = np.zeros((m.V, 3))
    args = [_c(theta, np.float64), _c(phi, np.float64), _c(phi, np.float64),
            _c(n, np.float64), _c(delta, np.float64), _c(cnt, np.int32)]
    lib().orc_shape_step_literal(ctypes.byref(m.c), *[_p(a) for a in args], ctypes.c_double(lambda_phi),
                                 ctypes.c_double(lambda_nbr), ctypes.c_double(lambda_w), _p(out))
    return out


class FrameResult(dict):
    pass


def track_frame(model, cam, params, theta, phi, phi_prev, depth=None, xyz=None, assoc=None, fp32=False):
    """Run one frame; theta/phi/phi_prev are updated in place (float64).

    assoc (test hook): int32 [n_iters, H*W] matches used instead of each
    iteration's own association (another implementation's choice at pixels
    whose candidates tie within rounding).

    fp32: run the float32 instantiation of the same source instead (a timing
    baseline at the GPU path's precision; its energies and step norm are not
    reported: NaN, and assoc_first stays -1).

    Returns dict(status, n_valid_px, n_assoc_px, n_obs_verts, energy_first,
    energy_last, step_norm_last, energies [n_iters], assoc_first [H*W])."""
    m = _model(model)
    n_it = int(params["n_iters"])
    dp = _c(params["do_pose"], np.uint8)
    ds = _c(params["do_shape"], np.uint8)
    act = params.get("active")
    act = None if act is None else _c(act, np.uint8)
    pr = _Params(float(params["tau"]), n_it, _p(dp), _p(ds), _p(act),
                 float(params["lambda_k"]), float(params["lambda_s"]),
                 float(params["lambda_phi"]), float(params["lambda_nbr"]),
                 float(params["lambda_t"]), float(params["lambda_w"]))
    for arr in (theta, phi, phi_prev):
        assert arr.dtype == np.float64 and arr.flags.c_contiguous
    c = _cam(cam)
    si = np.zeros(4, np.int32)
    sd = np.zeros(3)
    en = np.zeros(n_it)
    af = np.full(int(cam["width"]) * int(cam["height"]), -1, np.int32)
    d = None if depth is None else _c(depth, np.float32)
    x = None if xyz is None else _c(xyz, np.float32)
    ai = None
    if assoc is not None:
        ai = _c(assoc, np.int32).reshape(-1)
        assert ai.shape[0] == n_it * af.shape[0], "assoc must be [n_iters, H*W]"
    if fp32:
        assert assoc is None, "the float32 instantiation has no association hook"
        rc = lib().orc32_track_frame(ctypes.byref(m.c), ctypes.byref(c), ctypes.byref(pr), _p(theta),
                                     _p(phi), _p(phi_prev), _p(d), _p(x), _p(si))
        sd[:] = np.nan
        en[:] = np.nan
    else:
        rc = lib().orc_track_frame(ctypes.byref(m.c), ctypes.byref(c), ctypes.byref(pr), _p(theta),
                                   _p(phi), _p(phi_prev), _p(d), _p(x), _p(si), _p(sd), _p(en), _p(af), _p(ai))
    return FrameResult(status=int(rc), n_valid_px=int(si[1]), n_assoc_px=int(si[2]),
                       n_obs_verts=int(si[3]), energy_first=float(sd[0]),
                       energy_last=float(sd[1]), step_norm_last=float(sd[2]),
                       energies=en, assoc_first=af)
