"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks one oracle function against something other than itself:
closed forms, invariants, brute force, finite differences, forward-mode dual
numbers, or a library routine (numpy / scipy).  None of these tests needs a
GPU.
"""
import math

import numpy as np
import pytest
from scipy.linalg import cho_factor, cho_solve
from scipy.spatial.transform import Rotation

import oracle
from planted_cases import planted_cloud, planted_expectations
import synth


# ---------------------------------------------------------------------------
# helpers written independently of the oracle: homogeneous 4x4 matrices
# ---------------------------------------------------------------------------
def matrix_chain(model, theta):
    """World 4x4 of every joint: M_j = M_parent @ Offset_j @ Joint_j(theta_j)."""
    P = len(model["joint_parent"])
    M = []
    for j in range(P):
        off = np.eye(4)
        q = model["joint_offset"][j, :4].astype(float)
        off[:3, :3] = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        off[:3, 3] = model["joint_offset"][j, 4:]
        Jm = np.eye(4)
        ax = model["joint_axis"][j].astype(float)
        if model["joint_type"][j] == 0:
            Jm[:3, :3] = Rotation.from_rotvec(ax * theta[j]).as_matrix()
        else:
            Jm[:3, 3] = ax * theta[j]
        p = model["joint_parent"][j]
        M.append((np.eye(4) if p < 0 else M[p]) @ off @ Jm)
    return np.array(M)


def apply(M, x):
    return x @ M[:3, :3].T + M[:3, 3]


def one_hot(model):
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in model.items()}
    sl = m["skin_link"].copy()
    sw = m["skin_w"].copy()
    keep = np.argmax(sw, axis=1)
    new_l = np.full_like(sl, -1)
    new_w = np.zeros_like(sw)
    new_l[:, 0] = sl[np.arange(sl.shape[0]), keep]
    new_w[:, 0] = 1.0
    m["skin_link"], m["skin_w"] = new_l, new_w
    return m


def random_pose(body, rng, ang=0.4, trans=0.05):
    P = len(body.model["joint_parent"])
    return np.where(body.angular, rng.uniform(-ang, ang, P), rng.uniform(-trans, trans, P))


# ---------------------------------------------------------------------------
# Section 3.1: Eq. (1), (2) and the FK recursion
# ---------------------------------------------------------------------------
def test_fk_matches_homogeneous_matrix_chain(small_body, rng):
    m = small_body.model
    for _ in range(3):
        th = random_pose(small_body, rng)
        Hj, _ = oracle.fk(m, th)
        M = matrix_chain(m, th)
        pts = rng.normal(0, 0.5, (4, 3))
        for j in range(len(th)):
            for x in pts:
                T, _ = oracle.transform(Hj[j], x)
                np.testing.assert_allclose(T, apply(M[j], x), atol=1e-12)


def test_hinge_and_prismatic_closed_forms():
    # single hinge about a random axis through a pivot, then a prismatic
    rng = np.random.default_rng(77)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    ax2 = rng.normal(size=3)
    ax2 /= np.linalg.norm(ax2)
    model = dict(joint_parent=np.array([-1, 0], np.int32), joint_type=np.array([0, 1], np.int32),
                 joint_axis=np.array([ax, ax2], np.float32),
                 joint_offset=np.array([[1, 0, 0, 0, 0.3, -0.2, 1.0], [1, 0, 0, 0, 0, 0, 0]], np.float32),
                 link_joint=np.array([1], np.int32), rest_xyz=np.zeros((1, 3), np.float32),
                 faces=np.zeros((1, 3), np.int32), skin_link=np.zeros((1, 1), np.int32),
                 skin_w=np.ones((1, 1), np.float32), neighbors=None)
    axf = model["joint_axis"].astype(float)
    # the float32 axes are unit only to within rounding; a rotation about an
    # axis of length 1+e turns by up to e more than the closed form
    tol = 1e-12 + 4.0 * float(np.abs(np.linalg.norm(axf, axis=1) - 1.0).max()) * 4.0
    for th in (0.0, 0.7, -2.5, math.pi):
        Hj, _ = oracle.fk(model, np.array([th, 0.25]))
        # Eq. (1): real part cos(th/2) + z sin(th/2), offset composed in front
        x = rng.normal(size=3)
        T, _ = oracle.transform(Hj[0], x)
        R = Rotation.from_rotvec(axf[0] * th).as_matrix()
        t0 = model["joint_offset"][0, 4:].astype(float)
        np.testing.assert_allclose(T, R @ x + t0, rtol=0, atol=tol)
        # Eq. (2): translation by 0.25 along the second axis after the hinge
        T2, _ = oracle.transform(Hj[1], x)
        np.testing.assert_allclose(T2, R @ (x + 0.25 * axf[1]) + t0, rtol=0, atol=tol)


# ---------------------------------------------------------------------------
# Section 3.2: Eq. (3)-(5) skinning
# ---------------------------------------------------------------------------
def test_one_hot_skinning_is_the_link_rigid_motion(small_body, rng):
    m = one_hot(small_body.model)
    th = random_pose(small_body, rng)
    v, _ = oracle.skin(m, th)
    M = matrix_chain(m, th)
    M0 = matrix_chain(m, np.zeros_like(th))
    D = np.array([M[j] @ np.linalg.inv(M0[j]) for j in m["link_joint"]])
    x = m["rest_xyz"].astype(float)
    want = np.einsum("vij,vj->vi", D[m["skin_link"][:, 0], :3, :3], x) + D[m["skin_link"][:, 0], :3, 3]
    np.testing.assert_allclose(v, want, atol=1e-12)


def test_skinning_with_only_root_motion_is_rigid(small_body, rng):
    m = small_body.model
    th = np.zeros(len(m["joint_parent"]))
    th[:6] = [0.02, -0.03, 0.05, 0.3, -0.2, 0.1]
    phi = rng.normal(0, 0.004, (m["rest_xyz"].shape[0], 3))
    v, _ = oracle.skin(m, th, phi)
    M = matrix_chain(m, th)
    M0 = matrix_chain(m, np.zeros_like(th))
    G = M[5] @ np.linalg.inv(M0[5])
    np.testing.assert_allclose(v, apply(G, m["rest_xyz"].astype(float) + phi), atol=1e-12)


def test_blend_of_coaxial_rotations_is_the_mid_angle(rng):
    # two links driven by hinges about the same axis through the origin; a
    # 50/50 dual-quaternion blend rotates by the mean angle exactly
    model = dict(joint_parent=np.array([-1, -1], np.int32), joint_type=np.array([0, 0], np.int32),
                 joint_axis=np.array([[0, 0, 1], [0, 0, 1]], np.float32),
                 joint_offset=np.array([[1, 0, 0, 0, 0, 0, 0]] * 2, np.float32),
                 link_joint=np.array([0, 1], np.int32),
                 rest_xyz=np.array([[0.3, 0.1, 0.2]], np.float32), faces=np.zeros((1, 3), np.int32),
                 skin_link=np.array([[0, 1]], np.int32), skin_w=np.array([[0.5, 0.5]], np.float32),
                 neighbors=None)
    for a, b in ((0.2, 1.0), (-0.7, 0.4), (2.0, 2.9)):
        v, _ = oracle.skin(model, np.array([a, b]))
        R = Rotation.from_rotvec([0, 0, 0.5 * (a + b)]).as_matrix()
        np.testing.assert_allclose(v[0], R @ model["rest_xyz"][0].astype(float), atol=1e-12)


def test_blend_transform_is_scale_invariant_and_equivariant(rng):
    # T(cH, x) = T(H, x) and T(G H, x) = G T(H, x) for a unit G
    def rnd_unit():
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        t = rng.normal(size=3)
        tq = np.array([0, *t])
        return np.concatenate([q, 0.5 * qmul(tq, q)])

    def qmul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])

    def dqmul(A, B):
        return np.concatenate([qmul(A[:4], B[:4]), qmul(A[:4], B[4:]) + qmul(A[4:], B[:4])])

    for _ in range(20):
        H = 0.3 * rnd_unit() + 0.7 * rnd_unit()
        x = rng.normal(size=3)
        T, _ = oracle.transform(H, x)
        T2, _ = oracle.transform(3.7 * H, x)
        np.testing.assert_allclose(T2, T, atol=1e-12)
        G = rnd_unit()
        TG, _ = oracle.transform(dqmul(G, H), x)
        GT, _ = oracle.transform(G, T)
        np.testing.assert_allclose(TG, GT, atol=1e-12)


def test_transform_jacobian_matches_finite_differences(rng):
    for _ in range(10):
        H = rng.normal(size=8)
        x = rng.normal(size=3)
        _, J = oracle.transform(H, x)
        h = 1e-6
        for c in range(8):
            e = np.zeros(8)
            e[c] = h
            Tp, _ = oracle.transform(H + e, x)
            Tm, _ = oracle.transform(H - e, x)
            np.testing.assert_allclose(J[:, c], (Tp - Tm) / (2 * h), rtol=1e-6, atol=1e-8)


# ---------------------------------------------------------------------------
# vertex normals
# ---------------------------------------------------------------------------
def _flat_model(n=6):
    xs, ys = np.meshgrid(np.linspace(0, 0.1, n), np.linspace(0, 0.1, n))
    pts = np.stack([xs.ravel(), ys.ravel(), np.full(n * n, 1.0)], 1).astype(np.float32)
    faces = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = i * n + j, i * n + j + 1, (i + 1) * n + j, (i + 1) * n + j + 1
            faces += [(a, b, d), (a, d, c)]
    root = dict(joint_parent=np.array([-1], np.int32), joint_type=np.array([0], np.int32),
                joint_axis=np.array([[0, 0, 1]], np.float32),
                joint_offset=np.array([[1, 0, 0, 0, 0, 0, 0]], np.float32),
                link_joint=np.array([0], np.int32))
    return dict(root, rest_xyz=pts, faces=np.array(faces, np.int32),
                skin_link=np.zeros((n * n, 1), np.int32), skin_w=np.ones((n * n, 1), np.float32),
                neighbors=None)


def test_normals_of_a_plane_are_exact():
    m = _flat_model()
    _, n = oracle.skin(m, np.zeros(1))
    np.testing.assert_allclose(n, np.tile([0.0, 0.0, 1.0], (n.shape[0], 1)), atol=0)
    m2 = dict(m, faces=m["faces"][:, [0, 2, 1]].copy())
    _, n2 = oracle.skin(m2, np.zeros(1))
    np.testing.assert_allclose(n2, -n, atol=0)


def test_normals_point_outward_and_rotate_with_the_mesh(small_body, rng):
    m = small_body.model
    th = np.zeros(len(m["joint_parent"]))
    _, n = oracle.skin(m, th)
    # outward: within 25 degrees of the capsule's analytic outward direction
    cosang = np.einsum("ij,ij->i", n, small_body.outward)
    assert np.percentile(cosang, 1) > math.cos(math.radians(25))
    th[3:6] = [0.4, -0.3, 0.2]
    _, n2 = oracle.skin(m, th)
    M = matrix_chain(m, th)
    M0 = matrix_chain(m, np.zeros_like(th))
    R = (M[5] @ np.linalg.inv(M0[5]))[:3, :3]
    np.testing.assert_allclose(n2, n @ R.T, atol=1e-12)


# ---------------------------------------------------------------------------
# Section 4.1: projective association and averaging
# ---------------------------------------------------------------------------
def brute_association(cam, tau, v32, depth=None, xyz=None):
    """Exhaustive nearest in-image vertex, float32 arithmetic in the stated
    operation order, ties to the lower index."""
    f32 = np.float32
    W, H = cam["width"], cam["height"]
    fx, fy, cx, cy = (f32(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    v = v32.astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        fu = np.floor((fx * v[:, 0]) / v[:, 2] + cx + f32(0.5))
        fv = np.floor((fy * v[:, 1]) / v[:, 2] + cy + f32(0.5))
    cand = (v[:, 2] > f32(1e-3)) & (fu >= 0) & (fu < W) & (fv >= 0) & (fv < H)
    idx = np.flatnonzero(cand)
    if xyz is not None:
        P = xyz.reshape(-1, 3).astype(np.float32)
        valid = np.isfinite(P).all(1) & (P[:, 2] > 0)
    else:
        d = depth.reshape(-1).astype(np.float32)
        u = (np.arange(W * H) % W).astype(np.float32)
        vv = (np.arange(W * H) // W).astype(np.float32)
        valid = np.isfinite(d) & (d > 0)
        P = np.stack([((u - cx) * d) / fx, ((vv - cy) * d) / fy, d], 1).astype(np.float32)
    t2 = f32(tau) * f32(tau)
    out = np.full(W * H, -1, np.int32)
    C = v[idx]
    for k in np.flatnonzero(valid):
        dx = C[:, 0] - P[k, 0]
        dy = C[:, 1] - P[k, 1]
        dz = C[:, 2] - P[k, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        ok = d2 < t2
        if ok.any():
            d2m = np.where(ok, d2, np.inf)
            out[k] = idx[int(np.argmin(d2m))]
    return out


def test_association_equals_brute_force(tiny, rng):
    m = tiny.body.model
    cam = tiny.body.camera
    th = tiny.theta_true[0] * 0.5
    v, _ = oracle.skin(m, th)
    v32 = v.astype(np.float32)
    # planted exact ties: duplicate some vertices at higher indices
    dup = rng.choice(v32.shape[0], 40, replace=False)
    v32 = np.concatenate([v32, v32[dup]])
    # vertices behind the camera and outside the image are never candidates
    v32 = np.concatenate([v32, np.array([[0, 0, -0.5], [5.0, 0, 0.6], [0.01, 0.0, 0.0005]], np.float32)])
    depth = tiny.frames[0]
    a_grid = oracle.associate(cam, 0.10, v32, depth=depth)
    a_ob = oracle.associate(cam, 0.10, v32, depth=depth, brute=True)
    a_np = brute_association(cam, 0.10, v32, depth=depth)
    np.testing.assert_array_equal(a_grid, a_np)
    np.testing.assert_array_equal(a_ob, a_np)
    assert (a_np >= 0).sum() > 1000
    assert not np.isin(a_np, np.arange(2000, v32.shape[0])).any()


def test_association_ties_and_cutoff_on_a_handmade_cloud():
    cam = dict(width=8, height=6, fx=10.0, fy=10.0, cx=3.5, cy=2.5)
    v = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.1, 0.0, 1.0], [0.0, 0.0, 1.3]], np.float32)
    xyz = np.zeros((6, 8, 3), np.float32)
    xyz[2, 3] = [0.0, 0.0, 1.0]      # exact tie of vertices 0 and 1 -> 0
    xyz[2, 4] = [0.1, 0.0, 1.0]      # on vertex 2
    xyz[1, 1] = [0.0, 0.0, 1.2]      # 0.1 from vertex 3, 0.2 from 0 and 1
    xyz[0, 0] = [0.0, 0.0, 1.5]      # 0.2 from vertex 3: beyond tau = 0.15
    a = oracle.associate(cam, 0.15, v, xyz=xyz).reshape(6, 8)
    assert a[2, 3] == 0 and a[2, 4] == 2 and a[1, 1] == 3 and a[0, 0] == -1
    assert (a[xyz[..., 2] == 0] == -1).all()
    np.testing.assert_array_equal(a.ravel(), brute_association(cam, 0.15, v, xyz=xyz))


def test_averaging_matches_numpy(tiny):
    m = tiny.body.model
    cam = tiny.body.camera
    v, _ = oracle.skin(m, tiny.theta_true[0] * 0.5)
    a = oracle.associate(cam, 0.10, v.astype(np.float32), depth=tiny.frames[0])
    cnt, delta = oracle.average(cam, a, v, depth=tiny.frames[0])
    f32 = np.float32
    d = tiny.frames[0].reshape(-1)
    W = cam["width"]
    u = (np.arange(d.size) % W).astype(np.float32)
    vv = (np.arange(d.size) // W).astype(np.float32)
    P = np.stack([((u - f32(cam["cx"])) * d) / f32(cam["fx"]), ((vv - f32(cam["cy"])) * d) / f32(cam["fy"]), d], 1)
    sel = a >= 0
    c2 = np.bincount(a[sel], minlength=v.shape[0])
    s = np.zeros_like(v)
    np.add.at(s, a[sel], P[sel].astype(float) - v[a[sel]])
    np.testing.assert_array_equal(cnt, c2)
    ok = c2 > 0
    np.testing.assert_allclose(delta[ok], s[ok] / c2[ok, None], atol=1e-15)
    assert (delta[~ok] == 0).all()


# ---------------------------------------------------------------------------
# Section 4.2: residual, Jacobian, normal equations, damped step
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("blend", [0, 1], ids=["dq", "linear"])
@pytest.mark.parametrize("which", ["tiny", "body"])
def test_pose_jacobian_matches_dual_numbers_and_finite_differences(which, blend, tiny, small_body, rng):
    body = tiny.body if which == "tiny" else small_body
    m = oracle.Model(dict(body.model, blend=blend))
    th = random_pose(body, rng, 0.5, 0.05)
    phi = rng.normal(0, 0.004, (m.V, 3))
    v, n = oracle.skin(m, th, phi)
    cnt = (rng.random(m.V) < 0.7).astype(np.int32)
    delta = rng.normal(0, 0.01, (m.V, 3))
    ps = oracle.pose_system(m, th, phi, n, delta, cnt)
    obs = cnt > 0
    for k in range(m.P):
        e = np.zeros(m.P)
        e[k] = 1.0
        _, dv = oracle.skin_dual(m, th, e, phi)
        jad = -(n * dv).sum(1)
        np.testing.assert_allclose(ps["J"][obs, k], jad[obs], atol=1e-12)
        h = 1e-6
        vp, _ = oracle.skin(m, th + h * e, phi)
        vm, _ = oracle.skin(m, th - h * e, phi)
        # r_i = n.(p~ - v) with p~ and n frozen: dr/dtheta = -n.dv/dtheta
        jfd = -(n * (vp - vm)).sum(1) / (2 * h)
        np.testing.assert_allclose(ps["J"][obs, k], jfd[obs], rtol=1e-6, atol=1e-8)
    assert (ps["J"][~obs] == 0).all()
    np.testing.assert_allclose(ps["r"][obs], (n * delta).sum(1)[obs], atol=1e-15)


def test_offset_jacobian_is_the_blended_rotation(tiny, rng):
    """dv_i/dphi_i equals the rotation of the normalised blend (used for
    dr/dphi = -R^T n in Section 4.3); checked with dual numbers against
    finite differences."""
    m = oracle.Model(tiny.body.model)
    th = random_pose(tiny.body, rng, 0.5, 0.05)
    phi = rng.normal(0, 0.004, (m.V, 3))
    for c in range(3):
        dphi = np.zeros((m.V, 3))
        dphi[:, c] = 1.0
        _, dv = oracle.skin_dual(m, th, None, phi, dphi)
        h = 1e-6
        vp, _ = oracle.skin(m, th, phi + h * dphi)
        vm, _ = oracle.skin(m, th, phi - h * dphi)
        np.testing.assert_allclose(dv, (vp - vm) / (2 * h), atol=1e-8)
        # a rotation: columns have unit length
        if c == 0:
            np.testing.assert_allclose(np.linalg.norm(dv, axis=1), 1.0, atol=1e-12)


def test_normal_equations_equal_dense_products(small_body, rng):
    m = oracle.Model(small_body.model)
    th = random_pose(small_body, rng)
    phi = rng.normal(0, 0.003, (m.V, 3))
    _, n = oracle.skin(m, th, phi)
    cnt = (rng.random(m.V) < 0.5).astype(np.int32)
    delta = rng.normal(0, 0.01, (m.V, 3))
    ps = oracle.pose_system(m, th, phi, n, delta, cnt)
    J, r = ps["J"], ps["r"]
    np.testing.assert_allclose(ps["A"], J.T @ J, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ps["b"], J.T @ r, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ps["rr"], r @ r, rtol=1e-12)
    np.testing.assert_array_equal(ps["A"], ps["A"].T)
    assert np.linalg.eigvalsh(ps["A"]).min() > -1e-9
    # default pose prior: (lambda_s S)^2 on the diagonal and times Theta in b
    S = oracle.prior_weights(m)
    sk = small_body.model["skin_link"]
    swt = small_body.model["skin_w"]
    par = small_body.model["joint_parent"]
    lj = small_body.model["link_joint"]
    chains = []
    for l in range(len(lj)):
        c, j = set(), lj[l]
        while j >= 0:
            c.add(j)
            j = par[j]
        chains.append(c)
    for k in range(m.P):
        if k in chains[0]:
            assert S[k] == 0.0
            continue
        hit = sum(any(sk[i, q] >= 0 and swt[i, q] > 0 and k in chains[sk[i, q]] for q in range(m.K))
                  for i in range(m.V))
        assert S[k] == pytest.approx(hit / m.V, abs=0)
    ps2 = oracle.pose_system(m, th, phi, n, delta, cnt, lambda_s=0.7)
    np.testing.assert_allclose(ps2["A"] - ps["A"], np.diag((0.7 * S) ** 2), atol=1e-12)
    np.testing.assert_allclose(ps2["b"] - ps["b"], (0.7 * S) ** 2 * th, atol=1e-12)


def test_damped_cholesky_step_matches_scipy(small_body, rng):
    m = oracle.Model(small_body.model)
    th = random_pose(small_body, rng)
    _, n = oracle.skin(m, th)
    cnt = np.ones(m.V, np.int32)
    delta = rng.normal(0, 0.01, (m.V, 3))
    ps = oracle.pose_system(m, th, np.zeros((m.V, 3)), n, delta, cnt)
    A, b = ps["A"], ps["b"]
    x = oracle.lm_solve(A, b, 0.01)
    M = A + 0.01 * np.diag(np.diag(A))
    np.testing.assert_allclose(x, cho_solve(cho_factor(M), b), rtol=1e-9, atol=1e-12)
    # frozen parameters: an all-zero row/column and an inactive mask
    A2 = A.copy()
    A2[4, :] = 0
    A2[:, 4] = 0
    act = np.ones(m.P, np.uint8)
    act[10] = 0
    x2 = oracle.lm_solve(A2, b, 0.01, act)
    keep = np.array([k not in (4, 10) for k in range(m.P)])
    M2 = (A2 + 0.01 * np.diag(np.diag(A2)))[np.ix_(keep, keep)]
    np.testing.assert_allclose(x2[keep], np.linalg.solve(M2, b[keep]), rtol=1e-9, atol=1e-12)
    assert x2[4] == 0 and x2[10] == 0
    with pytest.raises(np.linalg.LinAlgError):
        oracle.lm_solve(-np.eye(3), np.ones(3), 0.01)


# ---------------------------------------------------------------------------
# Section 4.3: regularised per-vertex step
# ---------------------------------------------------------------------------
def test_shape_step_solves_each_vertex_system(tiny, rng):
    m = oracle.Model(tiny.body.model)
    th = random_pose(tiny.body, rng, 0.3, 0.02)
    phi = rng.normal(0, 0.003, (m.V, 3))
    phi_prev = phi + rng.normal(0, 0.001, (m.V, 3))
    _, n = oracle.skin(m, th, phi)
    cnt = (rng.random(m.V) < 0.6).astype(np.int32)
    delta = rng.normal(0, 0.005, (m.V, 3))
    lp, ln, lt, lw = 0.01, 1.0, 0.5, 0.1
    out = oracle.shape_step(m, th, phi, phi_prev, n, delta, cnt, lp, ln, lt, lw)
    # u_i = -(dv_i/dphi_i)^T n_i from dual numbers
    R = np.zeros((m.V, 3, 3))
    for c in range(3):
        dphi = np.zeros((m.V, 3))
        dphi[:, c] = 1.0
        _, dv = oracle.skin_dual(m, th, None, phi, dphi)
        R[:, :, c] = dv
    nb = tiny.body.model["neighbors"]
    for i in rng.choice(m.V, 200, replace=False):
        obs = cnt[i] > 0
        u = -(R[i].T @ n[i]) if obs else np.zeros(3)
        r = n[i] @ delta[i] if obs else 0.0
        g = u * r + lp * phi[i] + lt * (phi[i] - phi_prev[i]) + ln * (phi[i] - phi[nb[i]]).sum(0)
        A = np.outer(u, u) + (lp + lt + ln * 4) * np.eye(3)
        Md = A + lw * np.diag(np.diag(A))
        np.testing.assert_allclose(out[i], phi[i] - np.linalg.solve(Md, g), atol=1e-14)
    # with no data term and no neighbours/temporal weight, a closed form
    out2 = oracle.shape_step(m, th, phi, phi, n, delta, np.zeros(m.V, np.int32), lp, 0.0, 0.0, lw)
    np.testing.assert_allclose(out2, phi - phi / (1 + lw), atol=1e-15)


# ---------------------------------------------------------------------------
# whole-step properties
# ---------------------------------------------------------------------------
def _splat(body, th):
    v, n = oracle.skin(body.model, th)
    facing = (n * v).sum(1) < 0
    xyz, _ = synth.splat_points(v.astype(np.float32), facing.astype(np.uint8), body.camera)
    return xyz


def test_energy_invariant_under_a_rigid_motion_of_model_and_data(tiny, rng):
    m = tiny.body.model
    cam = tiny.body.camera
    xyz = _splat(tiny.body, tiny.theta_true[0] * 0.5)
    th = tiny.theta_true[0] * 0.3

    def energy(model, xyz_img):
        v, n = oracle.skin(model, th)
        a = oracle.associate(cam, 0.10, v.astype(np.float32), xyz=xyz_img, brute=True)
        cnt, delta = oracle.average(cam, a, v, xyz=xyz_img)
        return oracle.pose_system(model, th, np.zeros_like(v), n, delta, cnt)["rr"], a

    e0, a0 = energy(m, xyz)
    rot = Rotation.from_rotvec([0.02, -0.03, 0.01])
    t = np.array([0.004, -0.003, 0.002])
    m2 = dict(m)
    q = rot.as_quat()  # x y z w
    # compose G with the root offset (identity rotation, translation t0)
    t0 = m["joint_offset"][0, 4:].astype(float)
    off = np.zeros(7, np.float32)
    off[:4] = [q[3], q[0], q[1], q[2]]
    off[4:] = rot.apply(t0) + t
    jo = m["joint_offset"].copy()
    jo[0] = off
    m2["joint_offset"] = jo
    m2["rest_xyz"] = (rot.apply(m["rest_xyz"].astype(float)) + t).astype(np.float32)
    pts = xyz.reshape(-1, 3)
    valid = pts[:, 2] > 0
    moved = np.zeros_like(pts)
    moved[valid] = rot.apply(pts[valid].astype(float)) + t
    e1, a1 = energy(m2, moved.reshape(xyz.shape).astype(np.float32))
    assert (a0 == a1).mean() > 0.999
    assert e1 == pytest.approx(e0, rel=2e-3)


def test_vertex_splat_frame_is_a_fixed_point_and_attracts(tiny):
    body = tiny.body
    th_true = tiny.theta_true[0]
    xyz = _splat(body, th_true)
    P = len(th_true)
    n = 30
    prm = dict(tiny.params, n_iters=n, do_pose=np.ones(n, np.uint8), do_shape=np.zeros(n, np.uint8))
    # (a) stationary at the generating pose with Phi = 0, up to the float32
    # rounding of the splatted points (about 3e-8 m at 0.6 m)
    th = th_true.copy()
    phi = np.zeros((2000, 3))
    pp = phi.copy()
    r = oracle.track_frame(body.model, body.camera, dict(prm, n_iters=1), th, phi, pp, xyz=xyz)
    assert r["step_norm_last"] < 1e-6 and r["energy_first"] < 1e-11
    # shape steps leave Phi = 0 there too
    prm_s = dict(prm, n_iters=1, do_shape=np.ones(1, np.uint8))
    r = oracle.track_frame(body.model, body.camera, prm_s, th, phi, pp, xyz=xyz)
    assert np.abs(phi).max() < 1e-7
    # (b) pose-only Gauss-Newton from half the perturbation converges
    th = 0.5 * th_true
    r = oracle.track_frame(body.model, body.camera, prm, th, phi, pp, xyz=xyz)
    assert np.abs(th - th_true).max() < 1e-6
    assert r["energy_last"] < 1e-10


def test_converged_pose_is_stationary(tiny):
    """At a Gauss-Newton fixed point the gradient J^T r vanishes."""
    body = tiny.body
    depth = tiny.frames[0]
    th = 0.5 * tiny.theta_true[0]
    n = 25
    prm = dict(tiny.params, n_iters=n, do_pose=np.ones(n, np.uint8), do_shape=np.zeros(n, np.uint8))
    phi = np.zeros((2000, 3))
    pp = phi.copy()
    oracle.track_frame(body.model, body.camera, prm, th, phi, pp, depth=depth)
    v, nr = oracle.skin(body.model, th)
    a = oracle.associate(body.camera, 0.10, v.astype(np.float32), depth=depth)
    cnt, delta = oracle.average(body.camera, a, v, depth=depth)
    ps = oracle.pose_system(body.model, th, phi, nr, delta, cnt)
    scale = np.sqrt(np.diag(ps["A"]) * ps["rr"])
    assert (np.abs(ps["b"]) <= 1e-4 * scale).all()


def test_frame_driver_composes_the_steps(tiny):
    """One iteration of the frame driver equals the steps run by hand."""
    body = tiny.body
    cam = body.camera
    depth = tiny.frames[0]
    prm = dict(tiny.params, n_iters=1, do_pose=np.ones(1, np.uint8), do_shape=np.ones(1, np.uint8))
    th0 = 0.4 * tiny.theta_true[0]
    phi0 = np.random.default_rng(5).normal(0, 0.002, (2000, 3))
    prev = phi0 * 0.5
    th, phi, pp = th0.copy(), phi0.copy(), prev.copy()
    oracle.track_frame(body.model, cam, prm, th, phi, pp, depth=depth)
    v, n = oracle.skin(body.model, th0, phi0)
    a = oracle.associate(cam, prm["tau"], v.astype(np.float32), depth=depth)
    cnt, delta = oracle.average(cam, a, v, depth=depth)
    ps = oracle.pose_system(body.model, th0, phi0, n, delta, cnt)
    th1 = th0 - oracle.lm_solve(ps["A"], ps["b"], prm["lambda_k"])
    v1, n1 = oracle.skin(body.model, th1, phi0)
    delta1 = np.where(cnt[:, None] > 0, delta + (v - v1), delta)
    phi1 = oracle.shape_step(body.model, th1, phi0, prev, n1, delta1, cnt, prm["lambda_phi"],
                             prm["lambda_nbr"], prm["lambda_t"], prm["lambda_w"])
    np.testing.assert_array_equal(th, th1)
    np.testing.assert_array_equal(phi, phi1)
    np.testing.assert_array_equal(pp, phi1)
    # the association hook: given its own matches the driver is unchanged;
    # given another set it takes the step on those matches
    th2, phi2, pp2 = th0.copy(), phi0.copy(), prev.copy()
    oracle.track_frame(body.model, cam, prm, th2, phi2, pp2, depth=depth, assoc=a[None, :])
    np.testing.assert_array_equal(th2, th1)
    np.testing.assert_array_equal(phi2, phi1)
    a3 = a.copy()
    a3[np.flatnonzero(a3 >= 0)[::2]] = -1
    cnt3, delta3 = oracle.average(cam, a3, v, depth=depth)
    ps3 = oracle.pose_system(body.model, th0, phi0, n, delta3, cnt3)
    th3 = th0 - oracle.lm_solve(ps3["A"], ps3["b"], prm["lambda_k"])
    th4, phi4, pp4 = th0.copy(), phi0.copy(), prev.copy()
    oracle.track_frame(body.model, cam, prm, th4, phi4, pp4, depth=depth, assoc=a3[None, :])
    np.testing.assert_array_equal(th4, th3)
    assert np.abs(th4 - th1).max() > 1e-6


# ---------------------------------------------------------------------------
# blend sign rule (Section 3.2; Kavan et al.'s hemisphere alignment)
# ---------------------------------------------------------------------------
def _coaxial_pair(w0):
    """Two links on hinges about the same z axis through the origin, one
    vertex weighted w0 / 1 - w0 on them."""
    return dict(joint_parent=np.array([-1, -1], np.int32), joint_type=np.array([0, 0], np.int32),
                joint_axis=np.array([[0, 0, 1], [0, 0, 1]], np.float32),
                joint_offset=np.array([[1, 0, 0, 0, 0, 0, 0]] * 2, np.float32),
                link_joint=np.array([0, 1], np.int32),
                rest_xyz=np.array([[0.3, 0.1, 0.2]], np.float32), faces=np.zeros((1, 3), np.int32),
                skin_link=np.array([[0, 1]], np.int32), skin_w=np.array([[w0, 1.0 - w0]], np.float32),
                neighbors=None)


def test_blend_of_antipodal_hinges_takes_the_short_way():
    """Hinges at +3.0 and -3.0 rad: their rotation quaternions lie on
    opposite hemispheres (cos 3 < 0).  The rotations are 3.0 rad either way
    round, 0.28 rad apart through pi, so an even blend is the half turn about
    z.  Without the sign alignment the two quaternions' vector parts cancel
    and the blend is the identity."""
    m = _coaxial_pair(0.5)
    x = m["rest_xyz"][0].astype(float)
    v, _ = oracle.skin(m, np.array([3.0, -3.0]))
    np.testing.assert_allclose(v[0], Rotation.from_rotvec([0, 0, math.pi]).as_matrix() @ x, atol=1e-12)
    # -3.0 is the same rotation as 2 pi - 3.0; the blend of 3.0 and 2 pi - 3.0
    # on one hemisphere is their mean angle, pi, whatever the pivot
    for w0 in (0.3, 0.7):
        m = _coaxial_pair(w0)
        va, _ = oracle.skin(m, np.array([3.0, -3.0]))
        vb, _ = oracle.skin(m, np.array([3.0, 2 * math.pi - 3.0]))
        np.testing.assert_allclose(va, vb, atol=1e-12)


def test_skinning_is_invariant_to_a_full_turn_of_any_hinge(small_body, rng):
    """theta and theta + 2 pi give the same rotation and the negated
    quaternion (Eq. 1); the sign alignment makes the blended surface the same
    for every vertex, including those weighted on several links."""
    m = small_body.model
    th = random_pose(small_body, rng, 0.6, 0.03)
    v0, n0 = oracle.skin(m, th)
    multi = (m["skin_w"] > 0).sum(1) > 1
    assert multi.sum() > 100
    hinges = np.flatnonzero(small_body.angular)
    for k in rng.choice(hinges, 12, replace=False):
        t2 = th.copy()
        t2[k] += 2 * math.pi
        v1, n1 = oracle.skin(m, t2)
        np.testing.assert_allclose(v1, v0, atol=1e-12)
        np.testing.assert_allclose(n1, n0, atol=1e-9)


# ---------------------------------------------------------------------------
# area weighting of vertex normals (Section 4.1 uses the model's normal;
# reading: area-weighted face normals)
# ---------------------------------------------------------------------------
def _convex_mesh(rng, n=80):
    """Closed convex triangle mesh with irregular faces: the hull of random
    points near an ellipsoid, faces oriented outward."""
    from scipy.spatial import ConvexHull

    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = d * np.array([0.12, 0.08, 0.05]) * rng.uniform(0.9, 1.1, (n, 1)) + np.array([0.0, 0.0, 1.0])
    hull = ConvexHull(pts)
    keep = np.unique(hull.simplices)
    remap = -np.ones(n, np.int64)
    remap[keep] = np.arange(keep.size)
    P = pts[keep]
    F = remap[hull.simplices]
    c = P.mean(0)
    for f in range(F.shape[0]):
        a, b, e = P[F[f]]
        if np.dot(np.cross(b - a, e - a), a - c) < 0:
            F[f] = F[f][[0, 2, 1]]
    return P, F.astype(np.int32)


def test_vertex_normal_is_the_volume_gradient(rng):
    """On a closed mesh the sum over a vertex's faces of (v_b - v_a) x
    (v_c - v_a) is six times the gradient of the enclosed volume with
    respect to that vertex (the fan's edge terms cancel), so the
    area-weighted normal is the direction in which moving the vertex grows
    the volume fastest.  The volume comes from Qhull; it is linear in each
    vertex's coordinates, so central differences are exact up to rounding.
    Normalising each face normal before the sum (unit weights) fails this."""
    from scipy.spatial import ConvexHull

    P, F = _convex_mesh(rng)
    V = P.shape[0]
    model = dict(joint_parent=np.array([-1], np.int32), joint_type=np.array([0], np.int32),
                 joint_axis=np.array([[0, 0, 1]], np.float32),
                 joint_offset=np.array([[1, 0, 0, 0, 0, 0, 0]], np.float32),
                 link_joint=np.array([0], np.int32), rest_xyz=P.astype(np.float32), faces=F,
                 skin_link=np.zeros((V, 1), np.int32), skin_w=np.ones((V, 1), np.float32), neighbors=None)
    n = oracle.normals(model, P)
    facets = {tuple(sorted(f)) for f in F}
    h = 1e-5
    checked = 0
    for i in range(V):
        g = np.zeros(3)
        same = True
        for c in range(3):
            Pp, Pm = P.copy(), P.copy()
            Pp[i, c] += h
            Pm[i, c] -= h
            hp, hm = ConvexHull(Pp), ConvexHull(Pm)
            # a move that changes the hull's facets (nearly coplanar
            # neighbours) makes the volume non-linear: skip that vertex
            same = same and {tuple(sorted(f)) for f in hp.simplices} == facets
            same = same and {tuple(sorted(f)) for f in hm.simplices} == facets
            g[c] = (hp.volume - hm.volume) / (2 * h)
        if not same:
            continue
        checked += 1
        np.testing.assert_allclose(n[i], g / np.linalg.norm(g), atol=1e-7)
    assert checked >= 0.8 * V
    # the faces really are unequal (otherwise unit weights would pass too)
    areas = 0.5 * np.linalg.norm(np.cross(P[F[:, 1]] - P[F[:, 0]], P[F[:, 2]] - P[F[:, 0]]), axis=1)
    assert areas.max() > 3 * areas.min()


# ---------------------------------------------------------------------------
# per-vertex offset step derived from the energy (Section 4.3, Eq. 9 read as
# a sum of squared residuals)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("blend", [0, 1], ids=["dq", "linear"])
def test_shape_step_is_a_gauss_newton_step_on_the_vertex_energy(tiny, rng, blend):
    """Per vertex, with its neighbours' offsets, the mean associated point
    and the normal frozen, the energy is
        E_i(phi_i) = r_i(phi_i)^2 + l_phi |phi_i|^2
                     + l_N sum_n |phi_i - phi_n|^2 + l_T |phi_i - phi_i^prev|^2,
    r_i = n_i . (p~_i - v_i(phi_i)) with v_i from the skinning (pinned above).
    The step must be the damped Gauss-Newton step of E_i / 2: gradient g and
    Gauss-Newton matrix A = u u^T + alpha I, u = dr_i/dphi_i, both taken here
    by central differences of the energy and of r_i, then
    (A + l_w diag A) x = g and phi_i <- phi_i - x.  The same holds for
    the linear blend, whose d v_i / d phi_i is no longer a rotation."""
    m = oracle.Model(dict(tiny.body.model, blend=blend))
    th = random_pose(tiny.body, rng, 0.3, 0.02)
    phi = rng.normal(0, 0.003, (m.V, 3))
    prev = phi + rng.normal(0, 0.001, (m.V, 3))
    v, n = oracle.skin(m, th, phi)
    cnt = (rng.random(m.V) < 0.6).astype(np.int32)
    delta = rng.normal(0, 0.005, (m.V, 3))
    ptil = v + delta
    lp, ln, lt, lw = 0.01, 1.0, 0.5, 0.1
    out = oracle.shape_step(m, th, phi, prev, n, delta, cnt, lp, ln, lt, lw)
    nb = tiny.body.model["neighbors"]
    h = 1e-6
    # skinned positions with every vertex's offset moved by +-h along axis c
    # (each vertex's position depends on its own offset only)
    vp = [oracle.skin(m, th, phi + h * np.eye(3)[c])[0] for c in range(3)]
    vm = [oracle.skin(m, th, phi - h * np.eye(3)[c])[0] for c in range(3)]

    def energy(i, ph_i, vi):
        r = (n[i] @ (ptil[i] - vi)) if cnt[i] > 0 else 0.0
        e = r * r + lp * ph_i @ ph_i + lt * (ph_i - prev[i]) @ (ph_i - prev[i])
        for j in nb[i]:
            if j >= 0:
                e += ln * (ph_i - phi[j]) @ (ph_i - phi[j])
        return e, r

    for i in rng.choice(m.V, 150, replace=False):
        g = np.zeros(3)
        u = np.zeros(3)
        for c in range(3):
            e_p, r_p = energy(i, phi[i] + h * np.eye(3)[c], vp[c][i])
            e_m, r_m = energy(i, phi[i] - h * np.eye(3)[c], vm[c][i])
            g[c] = 0.25 * (e_p - e_m) / h
            u[c] = 0.5 * (r_p - r_m) / h
        alpha = lp + lt + ln * (nb[i] >= 0).sum()
        A = np.outer(u, u) + alpha * np.eye(3)
        x = np.linalg.solve(A + lw * np.diag(np.diag(A)), g)
        np.testing.assert_allclose(out[i], phi[i] - x, atol=1e-9)


# ---------------------------------------------------------------------------
# a rigid single link: point-to-plane least squares (Section 4.1 cites
# Chen and Medioni)
# ---------------------------------------------------------------------------
def test_rigid_link_gauss_newton_reaches_the_point_to_plane_least_squares_pose(tiny):
    """Every vertex on the root link (a rigid tube), association, mean points
    p~_i and normals n_i frozen at the start: the oracle's pose system and
    step, iterated with the offsets delta_i = p~_i - v_i(theta) recomputed
    from the skinning, converge to the minimiser of sum_i (n_i . (p~_i -
    v_i(theta)))^2 over the six root parameters, found here by scipy's
    least_squares on a 4x4-matrix model of the rigid motion."""
    from scipy.optimize import least_squares

    body = tiny.body
    m = one_hot(body.model)
    m["skin_link"][:, 0] = 0
    cam = body.camera
    th0 = 0.5 * tiny.theta_true[0]
    v0, n0 = oracle.skin(m, th0)
    a = oracle.associate(cam, 0.10, v0.astype(np.float32), depth=tiny.frames[0])
    cnt, d0 = oracle.average(cam, a, v0, depth=tiny.frames[0])
    obs = cnt > 0
    assert obs.sum() > 300
    ptil = v0 + d0
    th = th0.copy()
    for _ in range(60):
        v, _ = oracle.skin(m, th)
        ps = oracle.pose_system(m, th, np.zeros_like(v), n0, ptil - v, cnt)
        x = oracle.lm_solve(ps["A"], ps["b"], 1e-9)
        th = th - x
    assert np.abs(x).max() < 1e-12
    x_rest = m["rest_xyz"].astype(float)[obs]
    M0 = matrix_chain(m, np.zeros_like(th0))[5]

    def resid(q):
        t = th0.copy()
        t[:6] = q
        G = matrix_chain(m, t)[5] @ np.linalg.inv(M0)
        return (n0[obs] * (ptil[obs] - apply(G, x_rest))).sum(1)

    ls = least_squares(resid, th0[:6], xtol=1e-15, ftol=1e-15, gtol=1e-15)
    np.testing.assert_allclose(th[:6], ls.x, atol=1e-9)
    np.testing.assert_array_equal(th[6:], th0[6:])   # nothing observed moves the hinges


# ---------------------------------------------------------------------------
# noise-free rendered depth: convergence up to the sampling of the surface
# ---------------------------------------------------------------------------
def _converge_on_own_render(body, th_true, cam, params):
    v, _ = oracle.skin(body.model, th_true)
    depth = synth.raster_depth(v.astype(np.float32), body.model["faces"], cam)
    zwall = float(v[:, 2].max()) + 0.5
    depth = np.where(np.isfinite(depth), depth, np.float32(zwall)).astype(np.float32)
    n = 30
    prm = dict(params, n_iters=n, do_pose=np.ones(n, np.uint8), do_shape=np.zeros(n, np.uint8))
    th = 0.5 * th_true
    phi = np.zeros((v.shape[0], 3))
    r = oracle.track_frame(body.model, cam, prm, th, phi, phi.copy(), depth=depth)
    v2, _ = oracle.skin(body.model, th)
    return np.abs(th - th_true).max(), np.abs(v2 - v).max(), r["step_norm_last"]


def test_noise_free_rendered_depth_converges_within_the_mesh_sampling_bias(tiny):
    """Depth rendered (triangle z-buffer, no noise, no missing pixels) from
    the model's own surface at theta*.  Pixels sample the flat triangles
    between vertices while the residual measures them against the vertex's
    tangent plane, which lies off the triangles by about the sagitta
    s^2 / (8 R) of the vertex spacing s on a section of radius R (0.2 mm on
    the 2,000-vertex arm): pose-only Gauss-Newton from half the perturbation
    stops there, not at theta*.  The bias is below 0.5 mm per vertex and
    3e-3 rad per joint at 2,000 vertices and shrinks with the square of the
    spacing: at twice the sampling in each direction (7,994 vertices) it is
    below 0.3 times the first."""
    th_true = tiny.theta_true[0]
    cam = dict(width=320, height=240, fx=262.5, fy=262.5, cx=159.5, cy=119.5)
    ang0, vert0, step0 = _converge_on_own_render(synth.make_arm(), th_true, cam, tiny.params)
    ang1, vert1, step1 = _converge_on_own_render(synth.make_arm(74, 108), th_true, cam, tiny.params)
    assert step0 < 1e-6 and step1 < 1e-6          # converged
    assert vert0 < 5e-4 and ang0 < 3e-3
    assert vert1 < 0.3 * vert0 and ang1 < 0.3 * ang0


def test_planted_cloud_is_what_it_claims():
    """The planted cases on the CPU: the oracle's association of the cloud is
    brute force and each planted pixel gets the match its case is for."""
    cam, v32, xyz, where = planted_cloud()
    planted_expectations(cam, v32, xyz, where)
    # every point projects onto its own pixel (within rounding)
    P = xyz.reshape(-1, 3).astype(np.float64)
    k = np.flatnonzero(P[:, 2] > 0)
    uu = cam["fx"] * P[k, 0] / P[k, 2] + cam["cx"]
    vv = cam["fy"] * P[k, 1] / P[k, 2] + cam["cy"]
    assert np.abs(uu - k % cam["width"]).max() < 1e-3 and np.abs(vv - k // cam["width"]).max() < 1e-3


# ---------------------------------------------------------------------------
# Eq. (9) as printed: the negative result behind the least-squares reading
# ---------------------------------------------------------------------------
def _one_vertex():
    return dict(joint_parent=np.array([-1], np.int32), joint_type=np.array([0], np.int32),
                joint_axis=np.array([[0, 0, 1]], np.float32),
                joint_offset=np.array([[1, 0, 0, 0, 0, 0, 1.0]], np.float32),
                link_joint=np.array([0], np.int32), rest_xyz=np.array([[0.1, 0.2, 0.0]], np.float32),
                faces=np.zeros((1, 3), np.int32), skin_link=np.array([[0]], np.int32),
                skin_w=np.array([[1.0]], np.float32), neighbors=np.full((1, 4), -1, np.int32))


def test_literal_eq9_step_is_the_rank_one_closed_form_and_explodes():
    """One vertex, rest pose (R = I, so dr/dphi = -n), phi = 0: the printed
    system's step is x_k = r / ((3 + lam_w) j_k) with j = -n (the magnitude
    term adds nothing to j at phi = 0); a normal almost along x with small
    y, z parts turns a 1 mm residual into a step of tens of millimetres
    along z, while the reading's step, whose magnitude term adds lam_phi I
    to its 3x3 matrix, is at most the residual."""
    j = np.array([0.999, 0.04, 0.01])
    j /= np.linalg.norm(j)
    n = -j[None, :]
    r = 1e-3
    delta = r * n
    cnt = np.ones(1, np.int32)
    phi = np.zeros((1, 3))
    lw = 0.1
    out = oracle.shape_step_literal(_one_vertex(), np.zeros(1), phi, n, delta, cnt, 0.01, 0.0, lw)
    x = phi - out
    np.testing.assert_allclose(x[0], r / ((3 + lw) * j), rtol=1e-12)
    assert abs(x[0, 2]) > 0.03
    ours = oracle.shape_step(_one_vertex(), np.zeros(1), phi, phi, n, delta, cnt, 0.01, 0.0, 0.0, lw)
    assert np.linalg.norm(phi - ours) <= r


def test_literal_eq9_diverges_on_the_tiny_arm_where_the_reading_does_not(tiny):
    """Offset steps at the true pose of the tiny arm, re-associating each
    time: the printed form's offsets blow up in the first step; the
    reading's stay below a millimetre while the residual falls."""
    m, cam, prm = tiny.body.model, tiny.body.camera, tiny.params
    th = tiny.theta_true[0]
    for literal in (False, True):
        phi = np.zeros((2000, 3))
        rms = []
        for it in range(3):
            v, n = oracle.skin(m, th, phi)
            if not np.isfinite(v).all() or np.abs(v).max() > 1e3:
                break
            a = oracle.associate(cam, prm["tau"], v.astype(np.float32), depth=tiny.frames[0])
            cnt, delta = oracle.average(cam, a, v, depth=tiny.frames[0])
            rms.append(np.sqrt(np.mean(np.einsum("ij,ij->i", n, delta)[cnt > 0] ** 2)))
            if literal:
                phi = oracle.shape_step_literal(m, th, phi, n, delta, cnt, prm["lambda_phi"], prm["lambda_nbr"],
                                                prm["lambda_w"])
            else:
                phi = oracle.shape_step(m, th, phi, phi, n, delta, cnt, prm["lambda_phi"], prm["lambda_nbr"], 0.0,
                                        prm["lambda_w"])
        big = np.nanmax(np.abs(phi)) if np.isfinite(phi).any() else np.inf
        if literal:
            assert not np.isfinite(big) or big > 1.0      # metres
        else:
            assert big < 2e-3 and rms[-1] < rms[0]


# ---------------------------------------------------------------------------
# the linear variant of the blend (matrix linear blend skinning)
# ---------------------------------------------------------------------------
def test_linear_blend_equals_the_generators_matrix_skinning(small_body, rng):
    """Each link's rigid transform applied to the point, averaged with the
    weights: the input generator poses its ground truth this way with 4x4
    homogeneous matrices, an implementation of its own."""
    m = dict(small_body.model, blend=1)
    for _ in range(3):
        th = random_pose(small_body, rng, 0.6, 0.1)
        phi = rng.normal(0, 0.004, (m["rest_xyz"].shape[0], 3))
        v, _ = oracle.skin(m, th, phi)
        np.testing.assert_allclose(v, synth.pose_surface(m, th, phi), atol=1e-12)
    # and it differs from the dual-quaternion blend where links bend
    v_dq, _ = oracle.skin(small_body.model, th, phi)
    assert np.abs(v - v_dq).max() > 1e-4


def test_linear_and_dq_blends_agree_on_rigid_vertices(small_body, rng):
    m = one_hot(small_body.model)
    th = random_pose(small_body, rng, 0.6, 0.1)
    a, _ = oracle.skin(m, th)
    b, _ = oracle.skin(dict(m, blend=1), th)
    np.testing.assert_allclose(a, b, atol=1e-13)



def test_float32_instantiation_tracks_like_float64(tiny):
    """The float32 build of the same source (a CPU timing baseline at the
    GPU path's precision) follows the float64 frame on the tiny arm: same
    matches and status, joint angles within 1e-4 rad, offsets within 1e-6 m
    (float32 rounding through ten iterations)."""
    m, cam, prm = tiny.body.model, tiny.body.camera, tiny.params
    V = m["rest_xyz"].shape[0]
    out = []
    for fp32 in (False, True):
        th = tiny.theta0.copy()
        phi, prev = np.zeros((V, 3)), np.zeros((V, 3))
        r = oracle.track_frame(m, cam, prm, th, phi, prev, depth=tiny.frames[0], fp32=fp32)
        out.append((r, th, phi))
    (r64, th64, phi64), (r32, th32, phi32) = out
    assert r64["status"] == 0 and r32["status"] == 0
    assert r32["n_valid_px"] == r64["n_valid_px"]
    assert abs(r32["n_assoc_px"] - r64["n_assoc_px"]) <= 2
    assert np.abs(th32 - th64).max() < 1e-4
    assert np.abs(phi32 - phi64).max() < 1e-6
    assert not np.array_equal(th32, th64)   # it did run in another precision
