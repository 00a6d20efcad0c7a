"""Host-side tracking-quality measures (Section 5) against closed forms."""
import numpy as np

from paper_1711_07999_amd import metrics as M


def test_accuracy_curve_is_the_empirical_distribution():
    e = np.array([[0.01, 0.03], [0.03, 0.08]])
    t = np.array([0.0, 0.01, 0.02, 0.03, 0.05, 0.08, 0.1])
    np.testing.assert_array_equal(M.accuracy_curve(e, t), [0, 0.25, 0.25, 0.75, 0.75, 1.0, 1.0])


def test_auc_closed_forms():
    t = np.linspace(0, 0.1, 1001)
    assert M.curve_auc(t, M.accuracy_curve(np.zeros(10), t)) == 1.0
    assert M.curve_auc(t, M.accuracy_curve(np.full(10, 0.2), t)) == 0.0
    # errors uniform on [0, 0.1]: the curve is the identity on the range, area 1/2
    e = (np.arange(100000) + 0.5) / 100000 * 0.1
    assert abs(M.curve_auc(t, M.accuracy_curve(e, t)) - 0.5) < 1e-3


def test_rigid_segments_keep_the_largest_weight():
    model = dict(skin_link=np.array([[0, 1, -1], [2, 1, 0], [3, -1, -1]], np.int32),
                 skin_w=np.array([[0.4, 0.6, 0.0], [0.5, 0.5, 0.0], [1.0, 0.0, 0.0]], np.float32))
    r = M.rigid_segments(model)
    np.testing.assert_array_equal(r["skin_link"][:, 0], [1, 2, 3])
    np.testing.assert_array_equal(r["skin_w"].sum(1), [1, 1, 1])
    assert (r["skin_link"][:, 1:] == -1).all() and (r["skin_w"][:, 1:] == 0).all()


def _sphere(c, rad, n=40):
    th, ph = np.meshgrid(np.linspace(0.05, np.pi - 0.05, n), np.linspace(0, 2 * np.pi, 2 * n, endpoint=False))
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1).reshape(-1, 3)
    return np.asarray(c) + rad * d, d


def test_visibility_of_a_sphere_and_an_occluded_one():
    cam = dict(width=200, height=200, fx=200.0, fy=200.0, cx=99.5, cy=99.5)
    # vertex spacing about one pixel, as on the tracked meshes
    v1, n1 = _sphere((0, 0, 2.0), 0.3, 100)
    v2, n2 = _sphere((0, 0, 3.0), 0.1, 60)      # hidden behind the first
    vis = M.visible_vertices(np.vstack([v1, v2]), np.vstack([n1, n2]), cam, tol=0.01)
    cosv = -np.einsum("ij,ij->i", n1, v1) / np.linalg.norm(v1, axis=1)
    assert not vis[len(v1):].any()
    assert vis[:len(v1)][cosv <= 0].sum() == 0
    # away from the silhouette (where one pixel spans more than tol in depth)
    # every facing vertex is seen
    assert vis[:len(v1)][cosv > 0.5].all()


def test_reconstruction_error_to_a_plane():
    cam = dict(width=64, height=48, fx=60.0, fy=60.0, cx=31.5, cy=23.5)
    depth = np.full((48, 64), 2.0, np.float32)
    depth[:, :3] = 0.0
    # vertices 1 cm in front of the plane, facing the camera, near the centre
    xs = np.linspace(-0.3, 0.3, 7)
    v = np.array([[x, y, 1.99] for x in xs for y in xs])
    n = np.tile([0.0, 0.0, -1.0], (v.shape[0], 1))
    d = M.reconstruction_errors(v, n, depth, cam)
    assert d.shape[0] == v.shape[0]
    # nearest observed point: the plane 1 cm behind, offset by at most half a pixel sideways
    half = 0.5 * 2.0 / 60.0 * np.sqrt(2)
    assert (d >= 0.01 - 1e-12).all() and (d <= np.hypot(0.01, half) + 1e-12).all()


def test_mode_schedules():
    p, s = M.mode_schedule("full", 3, 5)
    assert p.tolist() == [1] * 5 and s.tolist() == [1] * 5
    assert M.mode_schedule("shape-match", 0, 5)[1].tolist() == [1] * 5
    assert M.mode_schedule("shape-match", 1, 5)[1].tolist() == [0] * 5
    assert M.mode_schedule("smooth-bind", 0, 5)[1].sum() == 0
    p, s = M.mode_schedule("paper-schedule", 0, 5)
    assert p.tolist() == [1] * 12 + [0, 0] and s.tolist() == [0] * 12 + [1, 1]
    p, s = M.mode_schedule("paper-schedule-linear", 3, 5)
    assert p.tolist() == [1] * 12 + [0, 0] and s.tolist() == [0] * 12 + [1, 1]
    assert M.model_for("paper-schedule-linear", {"blend": 0})["blend"] == 1
