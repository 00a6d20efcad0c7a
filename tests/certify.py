"""Certification of one GPU Gauss-Newton iteration against the float64
oracle, shared by the whole-frame and serving tests.

The GPU skins in float32 and the oracle in float64, so a pixel whose two
nearest vertices (or whose nearest vertex and the cutoff tau) are within the
vertices' rounding difference of each other can pick differently.  Such a
pixel has two correct matches: which one is taken depends on the rounding of
the surface.  An iteration is therefore checked in two parts:

1. every pixel whose match differs is certified as a near-tie on the
   oracle's float64 surface of the starting state: the two candidates'
   distances, or a distance and tau, differ by at most twice the largest
   difference between the GPU's float32 vertices and the float64 ones
   (eps), or the candidate's projection lies within eps f / z + 1e-5 px of
   the image border;
2. the oracle runs the iteration again taking the GPU's matches, and the
   GPU's pose and surface after the iteration are held to that result:
   1e-4 rad per joint angle, 1e-4 m per root translation and per vertex
   (both surfaces skinned by the oracle in float64).
"""
import numpy as np

import oracle

BAR_ANG, BAR_LIN = 1e-4, 1e-4


def points(cam, depth):
    """Back-projected points of a depth image, float32 order, as float64."""
    f32 = np.float32
    H, W = depth.shape
    u = np.arange(W, dtype=f32)[None, :]
    v = np.arange(H, dtype=f32)[:, None]
    d = depth.astype(f32)
    return np.stack([((u - f32(cam["cx"])) * d) / f32(cam["fx"]), ((v - f32(cam["cy"])) * d) / f32(cam["fy"]), d],
                    -1).reshape(-1, 3).astype(np.float64)


def uncertified(cam, tau, v64, eps, pts, a_g, a_o):
    """Indices of mismatched pixels that are not near-ties."""
    bad = []
    W, H = cam["width"], cam["height"]
    for k in np.flatnonzero(a_g != a_o):
        p = pts[k]
        ds = [np.linalg.norm(v64[i] - p) if i >= 0 else None for i in (a_g[k], a_o[k])]
        if ds[0] is not None and ds[1] is not None:
            if abs(ds[0] - ds[1]) <= 2 * eps:
                continue
        else:
            i = a_g[k] if a_g[k] >= 0 else a_o[k]
            dd = ds[0] if ds[0] is not None else ds[1]
            if abs(dd - tau) <= 2 * eps:
                continue
            x, y, z = v64[i]
            if z > 1e-3:
                uu = cam["fx"] * x / z + cam["cx"] + 0.5
                vv = cam["fy"] * y / z + cam["cy"] + 0.5
                edge = min(abs(uu), abs(uu - W), abs(vv), abs(vv - H))
                if edge <= 2 * eps * max(cam["fx"], cam["fy"]) / z + 1e-5:
                    continue
        bad.append(int(k))
    return bad


def check_iteration(model, cam, one, angular, th, phi, phi_prev, v32_start, depth, th_g, phi_g, a_g):
    """Certify one GPU iteration (params `one`, n_iters = 1) from the state
    (th, phi, phi_prev), whose float32 surface on the GPU was v32_start,
    which ended in (th_g, phi_g) with matches a_g.  Returns a dict with the
    mismatch count, the uncertified pixels, eps, the errors against the
    oracle on the GPU's matches (joint rad, root m, vertex m) and, for
    information, against the oracle's run on its own matches."""
    th_o, phi_o = th.copy(), phi.copy()
    r = oracle.track_frame(model, cam, one, th_o, phi_o, phi_prev.copy(), depth=depth)
    a_o = r["assoc_first"]
    v64, _ = oracle.skin(model, th, phi)
    eps = float(np.abs(v32_start.astype(np.float64) - v64).max())
    bad = uncertified(cam, float(one["tau"]), v64, eps, points(cam, depth), a_g, a_o)
    mis = int((a_g != a_o).sum())
    vg64, _ = oracle.skin(model, th_g, phi_g.astype(np.float64))
    vo64, _ = oracle.skin(model, th_o, phi_o)
    own = (float(np.abs(th_g - th_o)[angular].max()), float(np.abs(vg64 - vo64).max()))
    if mis and not bad:
        th_o, phi_o = th.copy(), phi.copy()
        oracle.track_frame(model, cam, one, th_o, phi_o, phi_prev.copy(), depth=depth, assoc=a_g[None, :])
        vo64, _ = oracle.skin(model, th_o, phi_o)
    d = np.abs(th_g - th_o)
    err = (float(d[angular].max()), float(d[~angular].max()) if (~angular).any() else 0.0,
           float(np.abs(vg64 - vo64).max()))
    ok = not bad and err[0] <= BAR_ANG and err[1] <= BAR_LIN and err[2] <= BAR_LIN
    return dict(mis=mis, bad=bad, eps=eps, err=err, own=own, ok=ok)


def describe(c):
    s = (f"assoc mismatches {c['mis']} ({len(c['bad'])} uncertified, eps {c['eps']:.1e} m); "
         f"joint {c['err'][0]:.1e} rad, root {c['err'][1]:.1e} m, vertex {c['err'][2]:.1e} m")
    if c["mis"]:
        s += f" (on the oracle's own matches: joint {c['own'][0]:.1e} rad, vertex {c['own'][1]:.1e} m)"
    return s


def truncated(prm, t):
    return dict(prm, n_iters=t, do_pose=np.asarray(prm["do_pose"])[:t].copy(),
                do_shape=np.asarray(prm["do_shape"])[:t].copy())


def walk_frame(T, trk, body, prm, th0, phi0, depth, log):
    """Per-iteration certification of one frame from (th0, phi0); returns the
    worst per-iteration differences and the list of failures."""
    m, cam = body.model, body.camera
    ang = body.angular
    n = int(prm["n_iters"])
    phi0 = phi0.astype(np.float32).astype(np.float64)
    th_prev, phi_prev_state = th0.copy(), phi0.copy()
    trk.reset(th0, phi0.astype(np.float32))
    v_gpu_prev = trk.state()[2]      # the GPU's float32 surface at the frame's start
    worst = [0.0, 0.0, 0.0]
    fails = []
    n_mis = 0
    for t in range(1, n + 1):
        trk.set_params(truncated(prm, t))
        trk.reset(th0, phi0.astype(np.float32))
        assert trk.frame(depth) == 0, T.track_last_error()
        th_g, phi_g, v_g, st = trk.state()
        a_g = T.track_dbg_get(trk.ctx, T.TRACK_BUF_ASSOC, (cam["height"] * cam["width"],), np.int32)
        # the oracle: one iteration (the flags of iteration t) from the GPU's
        # state before iteration t; phi_prev is the frame's start offsets
        one = dict(prm, n_iters=1, do_pose=np.asarray(prm["do_pose"])[t - 1:t].copy(),
                   do_shape=np.asarray(prm["do_shape"])[t - 1:t].copy())
        c = check_iteration(m, cam, one, ang, th_prev, phi_prev_state, phi0, v_gpu_prev, depth,
                                    th_g, phi_g, a_g)
        n_mis += c["mis"]
        worst = [max(x, y) for x, y in zip(worst, c["err"])]
        log(f"    it {t}: {describe(c)}")
        if c["bad"]:
            fails.append(f"iteration {t}: {len(c['bad'])} mismatches are not near-ties (first pixel {c['bad'][0]})")
        elif not c["ok"]:
            e = c["err"]
            fails.append(f"iteration {t}: joint {e[0]:.2e} rad, root {e[1]:.2e} m, vertex {e[2]:.2e} m")
        th_prev, phi_prev_state = th_g.copy(), phi_g.astype(np.float64)
        v_gpu_prev = v_g
    trk.set_params(prm)
    return worst, n_mis, fails
