"""Precision form: the split-bfloat16 Gram with float64 solves against the
float64 oracle, beside the plain float32 path.

Ten frames of the 50k-vertex body, each frame from the oracle's state at its
start (so the comparison measures one frame's arithmetic, not the drift of
weakly observed joints).  Per frame and per operand form: the largest
joint-angle error (rad), root-translation error (m) and vertex error (m)
against the oracle, and the oracle's own response to a 1e-6 perturbation of
the starting pose (the frame's amplification of rounding).  Prints the table
and a summary; every frame must stay inside the certified bound of the
end-to-end parity test.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_07999_amd import synth

pytestmark = pytest.mark.gpu

MODES = {"fp32": (0, 0), "fp32+fp64 solves": (0, 1), "bf16x3+fp64 solves": (1, 1), "bf16x6+fp64 solves": (2, 1)}
FLOOR = {(0, 0): (2e-3, 2e-3), (0, 1): (2e-3, 2e-3), (1, 1): (2e-2, 5e-3), (2, 1): (2e-3, 2e-3)}
PERTURB, GAIN = 1e-6, 10.0


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


def _oracle_frame(m, cam, prm, th, phi, depth):
    th, phi = th.copy(), phi.copy()
    oracle.track_frame(m, cam, prm, th, phi, phi.copy(), depth=depth)
    v, _ = oracle.skin(m, th, phi)
    return th, phi, v


def test_precision_forms_against_the_float64_oracle(T):
    w = synth.workload_human(n_frames=10)
    m, cam = w.body.model, w.body.camera
    V, P = m["rest_xyz"].shape[0], len(w.theta0)
    ang = w.body.angular
    trackers = {name: T.Tracker(m, cam, dict(w.params, gram_mode=g, pose_solve_fp64=f, shape_solve_fp64=f),
                                w.theta0) for name, (g, f) in MODES.items()}
    th_or, phi_or = w.theta0.copy(), np.zeros((V, 3))
    rows, failures = [], []
    try:
        _say("frame | oracle sensitivity (rad, m) | " + " | ".join(f"{k}: joint rad, root m, vertex m" for k in MODES))
        for f in range(len(w.frames)):
            phi_or = phi_or.astype(np.float32).astype(np.float64)
            prm = dict(w.params)
            th1, phi1, v1 = _oracle_frame(m, cam, prm, th_or, phi_or, w.frames[f])
            th2, _, v2 = _oracle_frame(m, cam, prm, th_or + PERTURB * np.random.default_rng(f).standard_normal(P),
                                       phi_or, w.frames[f])
            s_ang, s_v = np.abs(th2 - th1)[ang].max(), np.abs(v2 - v1).max()
            cells = []
            for name, (g, fp) in MODES.items():
                trk = trackers[name]
                trk.reset(th_or, phi_or.astype(np.float32))
                assert trk.frame(w.frames[f]) == 0, T.track_last_error()
                th_g, _, v_g, _ = trk.state()
                e = (np.abs(th_g - th1)[ang].max(), np.abs(th_g - th1)[~ang].max(), np.abs(v_g - v1).max())
                cells.append(e)
                f_ang, f_lin = FLOOR[(g, fp)]
                if not (e[0] <= max(f_ang, GAIN * s_ang) and e[2] <= max(f_lin, GAIN * s_v)):
                    failures.append((f, name))
            rows.append((s_ang, s_v, cells))
            _say(f"{f:5d} | {s_ang:.1e}, {s_v:.1e} | " +
                 " | ".join(f"{a:.1e}, {b:.1e}, {c:.1e}" for a, b, c in cells))
            th_or, phi_or = th1, phi1
    finally:
        for trk in trackers.values():
            trk.close()
    for q, name in enumerate(MODES):
        ea = np.array([r[2][q][0] for r in rows])
        ev = np.array([r[2][q][2] for r in rows])
        ok = np.mean((ea <= 1e-4) & (ev <= 1e-4))
        _say(f"{name:20s} joint rad median {np.median(ea):.1e} max {ea.max():.1e}; vertex m median "
             f"{np.median(ev):.1e} max {ev.max():.1e}; frames within 1e-4 rad and 0.1 mm: {ok:.0%}")
    assert not failures, failures
