"""The linear variant of the blend (TRACK_BLEND_LINEAR: matrix linear blend
skinning, each link's motion applied to the point and averaged with the
weights) through the C ABI against the oracle's linear blend: skinning, the
normal equations, the offset step, and whole frames certified iteration by
iteration, to the same bounds as the dual-quaternion path."""
import sys

import numpy as np
import pytest

import certify
import oracle
import synth

pytestmark = pytest.mark.gpu

ULP3 = np.spacing(np.float32(4.0))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_1711_07999_amd import track
    track.lib()
    return track


@pytest.fixture(scope="module")
def human():
    return synth.workload_human(n_frames=2)


def _case(name, tiny, human):
    w = tiny if name == "tiny" else human
    th = 0.5 * tiny.theta_true[0] if name == "tiny" else human.theta0
    return dict(w.body.model, blend=1), w.body.camera, dict(w.params), th, w.frames[0], w


def _assoc_inputs(m, cam, prm, th, depth, phi):
    v, _ = oracle.skin(m, th, phi)
    v32 = v.astype(np.float32)
    n32 = oracle.normals(m, v32.astype(np.float64)).astype(np.float32)
    a = oracle.associate(cam, prm["tau"], v32, depth=depth)
    cnt, delta = oracle.average(cam, a, v32.astype(np.float64), depth=depth)
    return v32, n32, cnt, delta.astype(np.float32)


@pytest.mark.parametrize("case", ["tiny", "human"])
def test_linear_skinning(T, tiny, human, case):
    _say(f"[blend] linear skinning {case}")
    m, cam, prm, th, _, _ = _case(case, tiny, human)
    V = m["rest_xyz"].shape[0]
    phi = np.random.default_rng(3).normal(0, 0.003, (V, 3)).astype(np.float32)
    trk = T.Tracker(m, cam, prm, th)
    try:
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_PHI, phi)
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_THETA, th)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_SKIN) == 0
        v = T.track_dbg_get(trk.ctx, T.TRACK_BUF_VERTS, (V, 3), np.float32)
    finally:
        trk.close()
    v_or, _ = oracle.skin(m, th, phi.astype(np.float64))
    assert np.abs(v - v_or).max() <= 16 * ULP3
    # and it is not the dual-quaternion blend
    v_dq, _ = oracle.skin(dict(m, blend=0), th, phi.astype(np.float64))
    assert np.abs(v_dq - v_or).max() > 1e-5


@pytest.mark.parametrize("case", ["tiny", "human"])
def test_linear_normal_equations(T, tiny, human, case):
    _say(f"[blend] linear normal equations {case}")
    m, cam, prm, th, depth, _ = _case(case, tiny, human)
    V, P = m["rest_xyz"].shape[0], len(th)
    phi = np.random.default_rng(11).normal(0, 0.002, (V, 3)).astype(np.float32)
    v32, n32, cnt, delta = _assoc_inputs(m, cam, prm, th, depth, phi.astype(np.float64))
    trk = T.Tracker(m, cam, prm, th)
    try:
        for buf, arr in ((T.TRACK_BUF_THETA, th), (T.TRACK_BUF_PHI, phi), (T.TRACK_BUF_VERTS, v32),
                         (T.TRACK_BUF_NORMALS, n32), (T.TRACK_BUF_COUNT, cnt.astype(np.int32)),
                         (T.TRACK_BUF_DELTA, delta)):
            T.track_dbg_set(trk.ctx, buf, arr)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_NORMAL_EQ) == 0
        G = T.track_dbg_get(trk.ctx, T.TRACK_BUF_GRAM, (P + 1, P + 1), np.float64)
    finally:
        trk.close()
    ps = oracle.pose_system(m, th, phi.astype(np.float64), n32.astype(np.float64), delta.astype(np.float64), cnt)
    J, r = ps["J"], ps["r"]
    aJ = np.abs(J)
    np.testing.assert_array_equal(G, G.T)
    assert (np.abs(G[:P, :P] - ps["A"]) <= 1e-4 * (aJ.T @ aJ) + 1e-12).all()
    assert (np.abs(G[:P, P] - ps["b"]) <= 1e-4 * (aJ.T @ np.abs(r)) + 1e-9).all()
    assert abs(G[P, P] - ps["rr"]) <= 1e-4 * ps["rr"] + 1e-12


@pytest.mark.parametrize("case", ["tiny", "human"])
def test_linear_offset_step(T, tiny, human, case):
    """Same inputs and bound as the dual-quaternion offset step:
    |dphi| <= 2e-4 |x| + 8 ulp(max|v|) / alpha_i."""
    _say(f"[blend] linear offset step {case}")
    m, cam, prm, th, depth, _ = _case(case, tiny, human)
    prm["lambda_t"] = 0.5
    V = m["rest_xyz"].shape[0]
    rng = np.random.default_rng(5)
    phi = rng.normal(0, 0.002, (V, 3)).astype(np.float32)
    prev = (phi + rng.normal(0, 0.001, (V, 3))).astype(np.float32)
    v32, n32, cnt, delta = _assoc_inputs(m, cam, prm, th, depth, phi.astype(np.float64))
    th2 = th + np.where(np.arange(len(th)) >= 6, 0.01, 0.001)
    trk = T.Tracker(m, cam, prm, th)
    try:
        for buf, arr in ((T.TRACK_BUF_PHI, phi), (T.TRACK_BUF_PHI_PREV, prev), (T.TRACK_BUF_VERTS, v32),
                         (T.TRACK_BUF_COUNT, cnt.astype(np.int32)), (T.TRACK_BUF_DELTA, delta),
                         (T.TRACK_BUF_THETA, th2)):
            T.track_dbg_set(trk.ctx, buf, arr)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_SHAPE) == 0
        phi_gpu = T.track_dbg_get(trk.ctx, T.TRACK_BUF_PHI, (V, 3), np.float32)
    finally:
        trk.close()
    v_new, n_new = oracle.skin(m, th2, phi.astype(np.float64))
    d_new = np.where(cnt[:, None] > 0, delta.astype(np.float64) + (v32.astype(np.float64) - v_new), delta)
    phi_or = oracle.shape_step(m, th2, phi.astype(np.float64), prev.astype(np.float64), n_new, d_new, cnt,
                               prm["lambda_phi"], prm["lambda_nbr"], prm["lambda_t"], prm["lambda_w"])
    x = np.abs(phi_or - phi).max(axis=1, keepdims=True)
    err = np.abs(phi_gpu - phi_or)
    nb = np.asarray(m["neighbors"])
    alpha = prm["lambda_phi"] + prm["lambda_t"] + prm["lambda_nbr"] * (nb >= 0).sum(axis=1)
    floor = 8 * float(np.spacing(np.float32(np.abs(v32).max()))) / alpha[:, None]
    assert (err <= 2e-4 * x + floor).all()


@pytest.mark.parametrize("case", ["tiny", "human"])
def test_linear_frame_certified_per_iteration(T, tiny, human, case):
    _say(f"[blend] linear frame {case}")
    m, cam, prm, th, depth, w = _case(case, tiny, human)
    th0 = w.theta0 if case == "human" else th

    class Body:
        pass

    body = Body()
    body.model, body.camera, body.angular = m, cam, w.body.angular
    trk = T.Tracker(m, cam, prm, th0)
    try:
        worst, _, fails = certify.walk_frame(T, trk, body, prm, th0, np.zeros((m["rest_xyz"].shape[0], 3)),
                                             depth, _say)
    finally:
        trk.close()
    _say(f"  worst per iteration: joint {worst[0]:.2e} rad, root {worst[1]:.2e} m, vertex {worst[2]:.2e} m")
    assert not fails, fails
