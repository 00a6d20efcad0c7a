"""Whole tracking frames on the GPU against the float64 oracle, certified
iteration by iteration.

Within a frame the two sides diverge only through the association: the GPU
skins in float32, the oracle in float64, so a pixel whose two nearest
vertices (or whose nearest vertex and the cutoff tau) are within the
vertices' rounding difference of each other can pick differently, and the
pose step then carries that difference into the next iteration.  The test
therefore walks the GPU's own trajectory one iteration at a time:

1. the GPU runs the frame truncated after t iterations (deterministic, so
   its iterations 1..t are those of the full frame); its state S_t and the
   association of iteration t are read back;
2. the oracle runs one iteration (the flags of iteration t) from the GPU's
   state S_{t-1};
3. every pixel whose match differs is certified as a near-tie on the
   oracle's float64 surface of S_{t-1}: the two candidates' distances, or a
   distance and tau, differ by at most twice the largest difference between
   the GPU's float32 vertices and the float64 ones (eps), or the candidate's
   projection lies within eps f / z + 1e-5 px of the image border;
4. where every mismatch is such a near-tie, both matches are correct
   results of the association (the rounding of the surface decides between
   them), so the oracle runs the same iteration again taking the GPU's
   matches, and the GPU's pose and surface after iteration t are held to
   that result: 1e-4 rad per joint angle, 1e-4 m per root translation and
   per vertex (both surfaces skinned by the oracle in float64).  The
   difference from the oracle's run on its own matches is printed beside it
   (one flipped pixel moves its vertex's offset step by up to tau).

Beside it the whole frame (all iterations, each side from the frame's start
state) is printed with the oracle's own response to a 1e-6 perturbation of
its start pose; a frame whose iterations all pass step 4 differs at the end
by the composition of its steps, which a weakly observed joint can amplify
(the printed response shows by how much).
"""
import sys

import numpy as np
import pytest

import certify
import oracle
import synth

pytestmark = pytest.mark.gpu

BAR_ANG, BAR_LIN = certify.BAR_ANG, certify.BAR_LIN


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
    return synth.workload_human(n_frames=3)


@pytest.fixture(scope="module")
def highres():
    return synth.workload_highres(n_frames=2)


def _whole_frame(T, trk, w, prm, th0, phi0, depth, log):
    """Whole frame from the same start on both sides, with the oracle's own
    response to a 1e-6 perturbation of the start pose (printed)."""
    m, cam = w.body.model, w.body.camera
    ang = w.body.angular
    trk.reset(th0, phi0.astype(np.float32))
    assert trk.frame(depth) == 0, T.track_last_error()
    th_g, phi_g, _, _ = trk.state()
    p0 = phi0.astype(np.float32).astype(np.float64)
    th_o, phi_o = th0.copy(), p0.copy()
    oracle.track_frame(m, cam, prm, th_o, phi_o, p0.copy(), depth=depth)
    th_p, phi_p = th0 + 1e-6 * np.random.default_rng(5).standard_normal(len(th0)), p0.copy()
    oracle.track_frame(m, cam, prm, th_p, phi_p, p0.copy(), depth=depth)
    vg, _ = oracle.skin(m, th_g, phi_g.astype(np.float64))
    vo, _ = oracle.skin(m, th_o, phi_o)
    vp, _ = oracle.skin(m, th_p, phi_p)
    dg, dp = np.abs(th_g - th_o), np.abs(th_p - th_o)
    log(f"    whole frame: GPU vs oracle joint {dg[ang].max():.1e} rad, vertex {np.abs(vg - vo).max():.1e} m; "
        f"oracle's response to 1e-6 rad: joint {dp[ang].max():.1e} rad, vertex {np.abs(vp - vo).max():.1e} m")
    return th_o, phi_o


def _run(T, w, prm, nframes):
    m, cam = w.body.model, w.body.camera
    V = m["rest_xyz"].shape[0]
    trk = T.Tracker(m, cam, prm, w.theta0)
    th, phi = w.theta0.copy(), np.zeros((V, 3))
    fails, worst_all = [], [0.0, 0.0, 0.0]
    try:
        for f in range(nframes):
            _say(f"  frame {f}")
            worst, n_mis, fl = certify.walk_frame(T, trk, w.body, prm, th, phi, w.frames[f], _say)
            worst_all = [max(a, b) for a, b in zip(worst_all, worst)]
            fails += [f"frame {f}, {x}" for x in fl]
            th, phi = _whole_frame(T, trk, w, prm, th, phi, w.frames[f], _say)
    finally:
        trk.close()
    _say(f"  worst per iteration: joint {worst_all[0]:.2e} rad, root {worst_all[1]:.2e} m, "
         f"vertex {worst_all[2]:.2e} m (bar {BAR_ANG:g} rad, {BAR_LIN:g} m)")
    return fails


MODES = {"fp32": (0, 0), "fp32+fp64 solves": (0, 1), "bf16x3+fp64 solves": (1, 1), "bf16x6+fp64 solves": (2, 1)}


@pytest.mark.parametrize("mode", list(MODES))
def test_human_frames_certified_per_iteration(T, human, mode):
    g, f = MODES[mode]
    _say(f"[frames] human-50k, {mode}")
    prm = dict(human.params, gram_mode=g, pose_solve_fp64=f, shape_solve_fp64=f)
    fails = _run(T, human, prm, 2)
    assert not fails, fails


@pytest.mark.parametrize("mode", ["smooth-bind", "paper-schedule"])
def test_human_schedules_certified_per_iteration(T, human, mode):
    """The pose-only schedule (smooth bind) and the paper's 12 pose then 2
    offset iterations per frame (Sections 4.2, 4.3), each iteration
    re-associating, held to the same per-iteration bar."""
    from paper_1711_07999_amd import metrics as M

    _say(f"[frames] human-50k, {mode}")
    dp, ds = M.mode_schedule(mode, 0, int(human.params["n_iters"]))
    prm = dict(human.params, n_iters=len(dp), do_pose=dp, do_shape=ds)
    fails = _run(T, human, prm, 1)
    assert not fails, fails


def test_joint_positions_match_a_matrix_chain(T, human):
    """track_joint_positions against the homogeneous-matrix forward
    kinematics of the input generator (Eq. 1, 2 and the chain of Section
    3.1 written independently)."""
    m = human.body.model
    trk = T.Tracker(m, human.body.camera, human.params, human.theta0)
    try:
        for f in range(len(human.frames)):
            th = human.theta_true[f]
            trk.reset(th)
            got = trk.joint_positions()
            want = synth.joint_matrices(m, th)[:, :3, 3]
            assert np.abs(got - want).max() < 1e-6
    finally:
        trk.close()


def test_highres_frames_certified_per_iteration(T, highres):
    _say("[frames] highres-200k (temporal weight 0.5, float64 pose solve)")
    fails = _run(T, highres, dict(highres.params), 2)
    assert not fails, fails


def test_tiny_frame_certified_per_iteration(T, tiny):
    _say("[frames] arm-2k, 10 iterations")
    fails = _run(T, tiny, dict(tiny.params), 1)
    assert not fails, fails
