"""Template refinement (Section 3.3) through the C ABI against the oracle,
then tracking on the refined template.

The synthetic low-resolution body (polygons, about 3,400 vertices, skin
weights on the 24 links) is refined by two rounds of Catmull-Clark
subdivision in the library and in the oracle: the same vertices and
triangles index by index (a quadrilateral whose two diagonals tie within
rounding may be split either way), positions within float32 rounding, the
same links per vertex (where weights tie within rounding, either order) and
weights within 1e-6.  The oracle's refined template (rounded to float32)
then serves as the tracked model: one frame rendered from a perturbed pose,
tracked on the GPU and certified iteration by iteration against the
oracle (tests/certify.py)."""
import sys

import numpy as np
import pytest

import certify
import synth
from oracle.subdivide import subdivide as oracle_subdivide

pytestmark = pytest.mark.gpu


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
def lowres():
    cam = dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5)
    return synth.make_lowres_body(cam, 2.6)


@pytest.fixture(scope="module")
def refined(lowres):
    lo = lowres
    return oracle_subdivide(lo["xyz"], lo["face_start"], lo["face_verts"], lo["skin_link"], lo["skin_w"], 2, 4)


def test_refinement_matches_the_oracle(T, lowres, refined):
    lo = lowres
    _say(f"[template] low-res {lo['xyz'].shape[0]} vertices, {len(lo['face_start']) - 1} polygons")
    x, tris, sl, sw = T.track_subdivide(lo["xyz"], lo["face_start"], lo["face_verts"], lo["skin_link"],
                                        lo["skin_w"], 2, 4)
    X, TT, L, W = refined
    _say(f"  refined: {x.shape[0]} vertices, {tris.shape[0]} triangles")
    assert x.shape == X.shape and tris.shape == TT.shape
    assert np.abs(x - X).max() <= 4 * np.finfo(np.float32).eps * np.abs(X).max()
    # triangles: per quadrilateral (2q, 2q + 1) identical, or a tie of its diagonals
    q = np.flatnonzero((tris != TT).any(1)) // 2
    for qq in np.unique(q):
        a, b = TT[2 * qq], TT[2 * qq + 1]
        corners = sorted(set(a) | set(b))
        assert sorted(set(tris[2 * qq]) | set(tris[2 * qq + 1])) == corners
        quad = [a[0], a[1], a[2], b[2]] if a[2] == b[1] else [a[0], a[1], b[1], b[2]]
        d1 = np.sum((X[quad[0]] - X[quad[2]]) ** 2)
        d2 = np.sum((X[quad[1]] - X[quad[3]]) ** 2)
        assert abs(d1 - d2) <= 1e-9 * max(d1, d2), (qq, d1, d2)
    _say(f"  quadrilaterals split along the other tied diagonal: {np.unique(q).size}")
    np.testing.assert_allclose(np.where(sl >= 0, sw, 0).sum(1), 1.0, atol=1e-6)
    for i in np.flatnonzero((sl != L).any(1)):
        # the same influences, ordered differently only where weights tie
        assert sorted(sl[i].tolist()) == sorted(L[i].tolist()), i
    order_g = np.argsort(sl, 1)
    order_o = np.argsort(L, 1)
    wg = np.take_along_axis(sw, order_g, 1)
    wo = np.take_along_axis(W, order_o, 1)
    assert np.abs(wg - wo).max() <= 1e-6


def _model(lo, refined):
    X, TT, L, W = refined
    m = dict(lo["model"])
    m["rest_xyz"] = X.astype(np.float32)
    m["faces"] = TT.astype(np.int32)
    m["skin_link"] = L.astype(np.int32)
    m["skin_w"] = W.astype(np.float32)
    m["neighbors"] = synth._neighbors4(m["rest_xyz"])
    return m


def test_frame_on_the_refined_template_is_certified(T, lowres, refined):
    m = _model(lowres, refined)
    cam = lowres["camera"]
    P = len(m["joint_parent"])
    ang = m["joint_type"] == synth.HINGE
    rng = np.random.default_rng(12)
    th_true = np.where(ang, rng.uniform(-0.08, 0.08, P), rng.uniform(-0.01, 0.01, P))
    depth = synth.render_frame(m, cam, synth.pose_surface(m, th_true), rng, 0.25, 0.002)
    th0 = th_true + np.where(ang, rng.uniform(-0.03, 0.03, P), rng.uniform(-0.01, 0.01, P))
    prm = synth.default_params(P, 5, 0.05, lambda_k=0.1)

    class Body:
        pass

    body = Body()
    body.model, body.camera, body.angular = m, cam, ang
    _say(f"[template] tracking one frame on the refined template ({m['rest_xyz'].shape[0]} vertices)")
    trk = T.Tracker(m, cam, prm, th0)
    try:
        worst, n_mis, fails = certify.walk_frame(T, trk, body, prm, th0, np.zeros((m["rest_xyz"].shape[0], 3)),
                                                 depth, _say)
    finally:
        trk.close()
    _say(f"  worst per iteration: joint {worst[0]:.2e} rad, root {worst[1]:.2e} m, vertex {worst[2]:.2e} m")
    assert not fails, fails
