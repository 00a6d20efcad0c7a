"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Per-pass tests inject identical inputs into both sides (the GPU through the
per-pass interface, the oracle through its functions) and compare outputs:
association indices and counts bit-exactly; floating point within bounds
derived from float32 arithmetic (stated per test).  Sizes: the tiny arm
(160x120, 2k vertices: several 8x8 tiles with a ragged tail of the vertex
chunks), a small body on a ragged 100x75 image (partial tiles) and the full
human workload (50k vertices, 640x480) in the launch configuration the
benchmark times.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from planted_cases import planted_cloud, planted_expectations

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
def human():
    return synth.workload_human(n_frames=4)


@pytest.fixture(scope="module")
def highres():
    return synth.workload_highres(n_frames=2)


@pytest.fixture(scope="module")
def ragged():
    cam = dict(width=100, height=75, fx=90.0, fy=90.0, cx=49.5, cy=37.0)
    body = synth.make_body(3001, cam, 2.6)
    rng = np.random.default_rng(7)
    P = len(body.model["joint_parent"])
    th = np.where(body.angular, rng.uniform(-0.1, 0.1, P), rng.uniform(-0.01, 0.01, P))
    depth = synth.render_frame(body.model, cam, synth.pose_surface(body.model, th), rng, 0.2, 0.002)
    return body, th, depth


def _cases(tiny, ragged, human, highres=None):
    b, th, d = ragged
    out = {
        "tiny": (tiny.body.model, tiny.body.camera, tiny.params, 0.5 * tiny.theta_true[0], tiny.frames[0]),
        "ragged": (b.model, b.camera, synth.default_params(len(th), 2, 0.05), 0.5 * th, d),
        "human": (human.body.model, human.body.camera, human.params, human.theta0, human.frames[0]),
    }
    if highres is not None:
        out["highres"] = (highres.body.model, highres.body.camera, highres.params, highres.theta0,
                          highres.frames[0])
    return out


ULP3 = np.spacing(np.float32(4.0))  # float32 spacing at the largest coordinate magnitudes here


@pytest.mark.parametrize("case", ["tiny", "ragged", "human", "highres"])
def test_skin_and_normals(T, tiny, ragged, human, highres, case):
    """Skinning at the same (theta, phi): float32 blend of float32-rounded
    link offsets, |dv| <= 16 ulp at 4 m.  Normals from the same float32
    vertices: float32 cross products and sums, |dn| <= 1e-5."""
    _say(f"[skin] {case}")
    m, cam, prm, th, _ = _cases(tiny, ragged, human, highres)[case]
    rng = np.random.default_rng(3)
    V = m["rest_xyz"].shape[0]
    phi = rng.normal(0, 0.003, (V, 3)).astype(np.float32)
    trk = T.Tracker(m, cam, prm, th)
    try:
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_PHI, phi)
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_THETA, th)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_SKIN) == 0
        v = T.track_dbg_get(trk.ctx, T.TRACK_BUF_VERTS, (V, 3), np.float32)
        v_or, _ = oracle.skin(m, th, phi.astype(np.float64))
        assert np.abs(v - v_or).max() <= 16 * ULP3
        v32 = v_or.astype(np.float32)
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_VERTS, v32)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_NORMALS) == 0
        n = T.track_dbg_get(trk.ctx, T.TRACK_BUF_NORMALS, (V, 3), np.float32)
        n_or = oracle.normals(m, v32.astype(np.float64))
        assert np.abs(n - n_or).max() <= 1e-5
    finally:
        trk.close()


def _bucket_cells(cam, v):
    """Cell (4x4 pixels, tile-major: 4 per 8x8 tile) of each float32 vertex
    by the library's bucket rule, -1 outside the image."""
    f32 = np.float32
    W, H = cam["width"], cam["height"]
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    with np.errstate(all="ignore"):
        u = np.floor((f32(cam["fx"]) * x) / z + f32(cam["cx"]) + f32(0.5))
        w = np.floor((f32(cam["fy"]) * y) / z + f32(cam["cy"]) + f32(0.5))
    ok = (z > f32(1e-3)) & (u >= 0) & (u < W) & (w >= 0) & (w < H)
    u = np.where(ok, u, 0).astype(np.int64)
    w = np.where(ok, w, 0).astype(np.int64)
    tile = (w // 8) * ((W + 7) // 8) + u // 8
    return np.where(ok, 4 * tile + 2 * ((w // 4) & 1) + ((u // 4) & 1), -1)


def _overflow(cam, v_layout, v_count):
    """Vertices of v_count that find their cell's region full when the
    regions were laid out from the counts of v_layout: tile t gets
    d + d/2 + 32 slots (d the largest count of the 3x3 tiles around it),
    each cell its count n + n/2 + 8 plus a quarter of the tile's remainder,
    the last cell the rest."""
    W, H = cam["width"], cam["height"]
    tx, ty = (W + 7) // 8, (H + 7) // 8
    ntiles = tx * ty
    ca = _bucket_cells(cam, v_layout)
    cnt = np.bincount(ca[ca >= 0], minlength=4 * ntiles).reshape(ntiles, 4)
    pad = np.pad(cnt.sum(1).reshape(ty, tx), 1)
    d = np.max([pad[1 + dy:1 + dy + ty, 1 + dx:1 + dx + tx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)], 0).reshape(-1)
    R = d + d // 2 + 32
    own = cnt + cnt // 2 + 8
    cap = own + ((R - own.sum(1)) // 4)[:, None]
    cap[:, 3] = R - cap[:, :3].sum(1)
    cb = _bucket_cells(cam, v_count)
    got = np.bincount(cb[cb >= 0], minlength=4 * ntiles).reshape(ntiles, 4)
    return int(np.maximum(got - cap, 0).sum())


@pytest.mark.parametrize("case", ["tiny", "ragged", "human", "highres"])
@pytest.mark.parametrize("source", ["depth", "xyz"])
def test_association_is_bit_exact(T, tiny, ragged, human, highres, case, source):
    """Same float32 vertices and frame: identical nearest-vertex index per
    pixel and identical counts; mean offsets within 1e-8 m (fixed-point sums
    quantised at 2^-32 m, float32 output).  Three associations in a row: the
    first finds no bucket layout (every vertex in the overflow list), the
    second the layout of the same surface (no overflow), the third the same
    layout for the surface moved by five pixels (cells that gained vertices
    overflow) -- the layout must not change the result."""
    _say(f"[assoc] {case} {source}")
    m, cam, prm, th, depth = _cases(tiny, ragged, human, highres)[case]
    v_or, _ = oracle.skin(m, th)
    v32 = v_or.astype(np.float32)
    # about five pixels across, three down
    px = float(np.median(v32[:, 2])) / cam["fx"]
    moved = (v32 + np.float32([5 * px, 3 * px, 0.0])).astype(np.float32)
    H, W = cam["height"], cam["width"]
    V = m["rest_xyz"].shape[0]
    assert _overflow(cam, v32, v32) == 0
    n_moved = _overflow(cam, v32, moved)
    _say(f"  {n_moved} vertices overflow on the moved surface")
    assert n_moved > 0
    trk = T.Tracker(m, cam, prm, th)
    try:
        if source == "xyz":
            # organised cloud with invalid pixels (z = 0, NaN) mixed in
            u = np.arange(W, dtype=np.float32)[None, :]
            vv = np.arange(H, dtype=np.float32)[:, None]
            d = depth.astype(np.float32)
            xyz = np.stack([((u - np.float32(cam["cx"])) * d) / np.float32(cam["fx"]),
                            ((vv - np.float32(cam["cy"])) * d) / np.float32(cam["fy"]), d], -1).astype(np.float32)
            xyz[::7, ::5] = np.nan
            T.track_dbg_set(trk.ctx, T.TRACK_BUF_XYZ, xyz)
            kw = dict(xyz=xyz)
        else:
            d = depth.copy()
            d[::9, ::4] = np.nan
            T.track_dbg_set(trk.ctx, T.TRACK_BUF_DEPTH, d)
            kw = dict(depth=d)
        for what, vs in (("no layout", v32), ("own layout", v32), ("moved surface", moved)):
            _say(f"  {what}")
            T.track_dbg_set(trk.ctx, T.TRACK_BUF_VERTS, vs)
            assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_ASSOCIATE) == 0
            a = T.track_dbg_get(trk.ctx, T.TRACK_BUF_ASSOC, (H * W,), np.int32)
            a_or = oracle.associate(cam, prm["tau"], vs, **kw)
            assert (a_or >= 0).sum() > 100
            np.testing.assert_array_equal(a, a_or, err_msg=what)
            cnt = T.track_dbg_get(trk.ctx, T.TRACK_BUF_COUNT, (V,), np.int32)
            delta = T.track_dbg_get(trk.ctx, T.TRACK_BUF_DELTA, (V, 3), np.float32)
            c_or, d_or = oracle.average(cam, a_or, vs.astype(np.float64), **kw)
            np.testing.assert_array_equal(cnt, c_or, err_msg=what)
            assert np.abs(delta - d_or).max() <= 1e-8, what
            # the same launch formed the surface's normals
            nrm = T.track_dbg_get(trk.ctx, T.TRACK_BUF_NORMALS, (V, 3), np.float32)
            n_or = oracle.normals(m, vs.astype(np.float64))
            assert np.abs(nrm - n_or).max() <= 1e-5, what
    finally:
        trk.close()


def test_skin_with_antipodal_influences(T, tiny):
    """Hinges past a half turn (3.5 and -3.4 rad) put the blend zones'
    influences on opposite quaternion hemispheres (cos(3.5 / 2) = -0.18), so
    the sign alignment of the blend decides every such vertex; adding a full
    turn to a hinge negates its quaternion and must leave the surface alone.
    Bound as for the skinning above: 16 ulp at 4 m."""
    _say("[skin] antipodal blend")
    m, cam, prm = tiny.body.model, tiny.body.camera, tiny.params
    V = m["rest_xyz"].shape[0]
    th = 0.5 * tiny.theta_true[0]
    th[6], th[7] = 3.5, -3.4
    multi = (m["skin_w"] > 0).sum(1) > 1
    assert multi.sum() > 100
    trk = T.Tracker(m, cam, prm, th)
    try:
        out = []
        for t in (th, th + 2 * math.pi * np.eye(len(th))[6]):
            T.track_dbg_set(trk.ctx, T.TRACK_BUF_THETA, t)
            assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_SKIN) == 0
            out.append(T.track_dbg_get(trk.ctx, T.TRACK_BUF_VERTS, (V, 3), np.float32))
    finally:
        trk.close()
    v_or, _ = oracle.skin(m, th)
    assert np.abs(out[0] - v_or).max() <= 16 * ULP3
    assert np.abs(out[1] - v_or).max() <= 16 * ULP3


def test_association_planted_ties_cutoff_and_non_candidates(T, tiny):
    _say("[assoc] planted cloud")
    cam, v32, xyz, where = planted_cloud()
    prm = dict(tiny.params, tau=0.125)
    trk = T.Tracker(tiny.body.model, cam, prm, tiny.theta0)
    try:
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_XYZ, xyz)
        T.track_dbg_set(trk.ctx, T.TRACK_BUF_VERTS, v32)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_ASSOCIATE) == 0
        a = T.track_dbg_get(trk.ctx, T.TRACK_BUF_ASSOC, (cam["height"] * cam["width"],), np.int32)
        cnt = T.track_dbg_get(trk.ctx, T.TRACK_BUF_COUNT, (2000,), np.int32)
    finally:
        trk.close()
    a_or = planted_expectations(cam, v32, xyz, where)
    np.testing.assert_array_equal(a, a_or)
    c_or, _ = oracle.average(cam, a_or, v32.astype(np.float64), xyz=xyz)
    np.testing.assert_array_equal(cnt, c_or)


def _assoc_inputs(m, cam, prm, th, depth, phi):
    v, n = oracle.skin(m, th, phi)
    v32 = v.astype(np.float32)
    n32 = oracle.normals(m, v32.astype(np.float64)).astype(np.float32)
    a = oracle.associate(cam, prm["tau"], v32, depth=depth)
    cnt, delta = oracle.average(cam, a, v32.astype(np.float64), depth=depth)
    return v32, n32, cnt, delta.astype(np.float32)


@pytest.mark.parametrize("case", ["tiny", "ragged", "human", "highres"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_normal_equations(T, tiny, ragged, human, highres, case, mode):
    """[J r]^T [J r] from identical (theta, phi, v, n, c, delta).
    float32 rows and MFMA accumulation:
      |dA_kl| <= 1e-4 (|J|^T|J|)_kl,  |db_k| <= 1e-4 (|J|^T|r|)_k + 1e-9,
      |d rr| <= 1e-4 rr.
    The split-bfloat16 forms carry about 2^-17 (hi/lo) and 2^-24 (hi/mid/lo)
    relative error per product, inside the same bound."""
    _say(f"[normal_eq] {case} mode={mode}")
    m, cam, prm, th, depth = _cases(tiny, ragged, human, highres)[case]
    prm = dict(prm, gram_mode=mode)
    V, P = m["rest_xyz"].shape[0], len(th)
    rng = np.random.default_rng(11)
    phi = rng.normal(0, 0.002, (V, 3)).astype(np.float32)
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
    ps = oracle.pose_system(m, th, phi.astype(np.float64), n32.astype(np.float64),
                            delta.astype(np.float64), cnt)
    J, r = ps["J"], ps["r"]
    aJ = np.abs(J)
    np.testing.assert_array_equal(G, G.T)
    assert (np.abs(G[:P, :P] - ps["A"]) <= 1e-4 * (aJ.T @ aJ) + 1e-12).all()
    assert (np.abs(G[:P, P] - ps["b"]) <= 1e-4 * (aJ.T @ np.abs(r)) + 1e-9).all()
    assert abs(G[P, P] - ps["rr"]) <= 1e-4 * ps["rr"] + 1e-12


def _blended_everywhere(m):
    """The same body with every vertex also weighted (lightly) on both hands
    and both feet: every pair of joints is then coupled, the tree form of the
    solve has no front that fits, and the dense form is taken."""
    m = dict(m)
    links, w = m["skin_link"].copy(), m["skin_w"].copy()
    far = [10, 15, 19, 23]
    for q in range(4):
        put = w[:, q] == 0.0
        links[put, q] = far[q]
        w[put, q] = 1e-3
    m["skin_link"], m["skin_w"] = links, (w / w.sum(1, keepdims=True)).astype(np.float32)
    return m


@pytest.mark.parametrize("fp64", [0, 1])
@pytest.mark.parametrize("form", ["tree", "dense", "dense-pattern"])
def test_pose_step(T, human, fp64, form, monkeypatch):
    """The damped Cholesky step on the GPU's own Gram matrix equals the
    oracle's solve of that matrix (float64: 1e-9 relative to |x|; float32:
    1e-4 relative -- the damped 75x75 system has condition number about 130
    once its diagonal is scaled to one, which a Cholesky factorisation does
    implicitly, so float32 carries about 130 x 6e-8 = 8e-6).  Forms:
    the tree-ordered factorisation (the default for the body), the dense
    one forced by TRACK_DENSE_SOLVE=1, and the dense one chosen because the
    skin couples every pair of joints."""
    _say(f"[pose_step] fp64={fp64} form={form}")
    m, cam, prm, th, depth = (human.body.model, human.body.camera, dict(human.params, pose_solve_fp64=fp64),
                              human.theta0, human.frames[0])
    if form == "dense":
        monkeypatch.setenv("TRACK_DENSE_SOLVE", "1")
    if form == "dense-pattern":
        m = _blended_everywhere(m)
    V, P = m["rest_xyz"].shape[0], len(th)
    phi = np.zeros((V, 3), np.float32)
    v32, n32, cnt, delta = _assoc_inputs(m, cam, prm, th, depth, phi.astype(np.float64))
    trk = T.Tracker(m, cam, prm, th)
    monkeypatch.delenv("TRACK_DENSE_SOLVE", raising=False)
    try:
        for buf, arr in ((T.TRACK_BUF_THETA, th), (T.TRACK_BUF_VERTS, v32), (T.TRACK_BUF_NORMALS, n32),
                         (T.TRACK_BUF_COUNT, cnt.astype(np.int32)), (T.TRACK_BUF_DELTA, delta)):
            T.track_dbg_set(trk.ctx, buf, arr)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_NORMAL_EQ) == 0
        G = T.track_dbg_get(trk.ctx, T.TRACK_BUF_GRAM, (P + 1, P + 1), np.float64)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_POSE_STEP) == 0
        step = T.track_dbg_get(trk.ctx, T.TRACK_BUF_STEP, (P,), np.float64)
        th_new = T.track_dbg_get(trk.ctx, T.TRACK_BUF_THETA, (P,), np.float64)
    finally:
        trk.close()
    # the library holds the damping constant in float32
    x = oracle.lm_solve(G[:P, :P], G[:P, P], float(np.float32(prm["lambda_k"])))
    tol = 1e-9 if fp64 else 1e-4
    _say(f"  step difference {np.abs(step - x).max() / np.abs(x).max():.2e} relative")
    assert np.abs(step - x).max() <= tol * np.abs(x).max()
    np.testing.assert_allclose(th_new, th - step, rtol=0, atol=1e-15)


@pytest.mark.parametrize("case", ["tiny", "human"])
@pytest.mark.parametrize("fp64", [0, 1])
def test_shape_step(T, tiny, human, case, fp64):
    """One offset step from identical inputs.  The GPU re-skins at theta in
    float32, so its normals carry ~ulp(v)/edge relative error (about 1e-4 on
    the 5 mm edges of the human mesh) and its residuals ~8 ulp(v); bound
    |dphi| <= 2e-4 |x| + 8 ulp(max|v|) / alpha_i with x the oracle's
    per-vertex step and alpha_i the vertex's regulariser weight."""
    _say(f"[shape] {case} fp64={fp64}")
    if case == "tiny":
        m, cam, prm, th, depth = (tiny.body.model, tiny.body.camera, dict(tiny.params), 0.5 * tiny.theta_true[0],
                                  tiny.frames[0])
        prm["lambda_t"] = 0.5
    else:
        m, cam, prm, th, depth = (human.body.model, human.body.camera, dict(human.params, lambda_t=0.5),
                                  human.theta0, human.frames[0])
    prm["shape_solve_fp64"] = fp64
    V = m["rest_xyz"].shape[0]
    rng = np.random.default_rng(5)
    phi = rng.normal(0, 0.002, (V, 3)).astype(np.float32)
    prev = (phi + rng.normal(0, 0.001, (V, 3))).astype(np.float32)
    v32, n32, cnt, delta = _assoc_inputs(m, cam, prm, th, depth, phi.astype(np.float64))
    th2 = th + np.where(np.arange(len(th)) >= 6, 0.01, 0.001)  # a pose step happened
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
    # rounding floor: the residual carries ~8 ulp of the float32 vertex
    # coordinates and enters the step divided by the regulariser weight
    nb = np.asarray(m["neighbors"])
    alpha = prm["lambda_phi"] + prm["lambda_t"] + prm["lambda_nbr"] * (nb >= 0).sum(axis=1)
    floor = 8 * float(np.spacing(np.float32(np.abs(v32).max()))) / alpha[:, None]
    bad = np.flatnonzero((err > 2e-4 * x + floor).any(axis=1))
    worst = int(np.argmax(err.max(axis=1) / (x[:, 0] + 1e-12)))
    assert bad.size == 0, (f"{bad.size} vertices, worst {worst}: err {err[worst].max():.3e} step {x[worst, 0]:.3e} "
                           f"count {cnt[worst]} |n| {np.linalg.norm(n_new[worst]):.3f}")


def test_runs_are_bit_identical_and_checkpoints_resume(T, human):
    _say("[determinism]")
    m, cam, prm = human.body.model, human.body.camera, human.params
    V, P = m["rest_xyz"].shape[0], len(human.theta0)
    outs = []
    for _ in range(2):
        trk = T.Tracker(m, cam, prm, human.theta0)
        for f in range(3):
            assert trk.frame(human.frames[f]) == 0
        outs.append(trk.state(want_verts=False)[:2])
        trk.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    # checkpoint after frame 1, resume in a fresh context
    trk = T.Tracker(m, cam, prm, human.theta0)
    assert trk.frame(human.frames[0]) == 0
    th_ck, phi_ck, _, _ = trk.state(want_verts=False)
    trk.close()
    trk = T.Tracker(m, cam, prm, th_ck, phi_ck)
    for f in (1, 2):
        assert trk.frame(human.frames[f]) == 0
    th2, phi2, _, _ = trk.state(want_verts=False)
    trk.close()
    np.testing.assert_array_equal(th2, outs[0][0])
    np.testing.assert_array_equal(phi2, outs[0][1])


def test_health_check_rejects_bad_frames_and_keeps_state(T, tiny):
    _say("[health]")
    m, cam, prm = tiny.body.model, tiny.body.camera, tiny.params
    th0 = 0.5 * tiny.theta_true[0]
    trk = T.Tracker(m, cam, prm, th0)
    try:
        before = trk.state()
        H, W = cam["height"], cam["width"]
        for bad in (np.zeros((H, W), np.float32), np.full((H, W), np.nan, np.float32),
                    np.full((H, W), 25.0, np.float32)):
            rc = trk.frame(bad)
            assert rc == T.TRACK_E_LOST, (rc, T.track_last_error())
            after = trk.state()
            np.testing.assert_array_equal(after[0], before[0])
            np.testing.assert_array_equal(after[1], before[1])
            assert after[3]["status"] == T.TRACK_E_LOST
        assert trk.frame(tiny.frames[0]) == 0
    finally:
        trk.close()


def test_vertex_splat_frame_converges(T, tiny):
    """Pose-only Gauss-Newton on a frame splatted from the model's own
    vertices at theta*: from half the perturbation the float32 GPU path
    reaches theta* to 1e-4."""
    _say("[splat]")
    m, cam = tiny.body.model, tiny.body.camera
    th_true = tiny.theta_true[0]
    v, n = oracle.skin(m, th_true)
    xyz, _ = synth.splat_points(v.astype(np.float32), ((n * v).sum(1) < 0).astype(np.uint8), cam)
    k = 30
    prm = dict(tiny.params, n_iters=k, do_pose=np.ones(k, np.uint8), do_shape=np.zeros(k, np.uint8))
    trk = T.Tracker(m, cam, prm, 0.5 * th_true)
    try:
        assert trk.frame_xyz(xyz) == 0, T.track_last_error()
        th = trk.state(want_verts=False)[0]
    finally:
        trk.close()
    assert np.abs(th - th_true).max() < 1e-4


@pytest.mark.parametrize("fp64", [0, 1])
def test_pose_step_with_an_inactive_joint(T, tiny, fp64):
    """Tiny arm with its last hinge masked inactive (6 root + 1 hinge = 7
    DoF): the masked step is exactly zero and the rest equals the oracle's
    solve of the GPU's Gram matrix with the same mask."""
    _say(f"[pose_step masked] fp64={fp64}")
    m, cam = tiny.body.model, tiny.body.camera
    P = len(tiny.theta0)
    active = np.ones(P, np.uint8)
    active[-1] = 0
    prm = dict(tiny.params, active=active, pose_solve_fp64=fp64)
    th = 0.5 * tiny.theta_true[0]
    phi = np.zeros((2000, 3), np.float32)
    v32, n32, cnt, delta = _assoc_inputs(m, cam, prm, th, tiny.frames[0], phi.astype(np.float64))
    trk = T.Tracker(m, cam, prm, th)
    try:
        for buf, arr in ((T.TRACK_BUF_THETA, th), (T.TRACK_BUF_VERTS, v32), (T.TRACK_BUF_NORMALS, n32),
                         (T.TRACK_BUF_COUNT, cnt.astype(np.int32)), (T.TRACK_BUF_DELTA, delta)):
            T.track_dbg_set(trk.ctx, buf, arr)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_NORMAL_EQ) == 0
        G = T.track_dbg_get(trk.ctx, T.TRACK_BUF_GRAM, (P + 1, P + 1), np.float64)
        assert T.track_dbg_run(trk.ctx, T.TRACK_PASS_POSE_STEP) == 0
        step = T.track_dbg_get(trk.ctx, T.TRACK_BUF_STEP, (P,), np.float64)
    finally:
        trk.close()
    x = oracle.lm_solve(G[:P, :P], G[:P, P], float(np.float32(prm["lambda_k"])), active)
    assert step[-1] == 0.0
    tol = 1e-9 if fp64 else 1e-4
    assert np.abs(step - x).max() <= tol * np.abs(x).max()
