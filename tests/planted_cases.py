"""A hand-built association case shared by the oracle's pins and the GPU
parity tests: planted exact ties, the cutoff, and vertices that are never
candidates, on an organised point cloud whose points lie on their pixels'
rays."""
import numpy as np

import oracle


def _backproject(cam, pu, pv, d):
    """The point of pixel (pu, pv) at depth d, in the float32 order of a
    depth image's back-projection (so it projects onto the pixel's centre)."""
    f32 = np.float32
    d = f32(d)
    return np.array([((f32(pu) - f32(cam["cx"])) * d) / f32(cam["fx"]),
                     ((f32(pv) - f32(cam["cy"])) * d) / f32(cam["fy"]), d], np.float32)


def planted_cloud():
    """A hand-built association case on the tiny arm's 160x120 camera with
    tau = 0.125 m (exact in binary).  Every point lies on its own pixel's ray,
    as the back-projection of a depth image does (the search is bounded
    around the pixel).  2,000 vertices are scattered in front of the camera
    at z in [0.6, 1.4] and points near them fill rows 16 and below; the
    planted cases sit at z >= 2 in rows 0..15 (or on the image border), at
    least 0.14 m from every other case's vertices:
      (a) exact ties: vertices 1500..1511 are copies of vertices 0..11 with a
          point 1 mm in front of each; pairs placed 2^-7 m in front of and
          behind a point (z = 2.05078125 makes every coordinate exact);
      (b) never candidates, each with a point closer than tau: vertices
          behind the camera, at z = 0, at exactly z_near = 1e-3 and one float
          below it (points at depth 0.01), and one projecting to u = -0.75;
      (c) vertices projecting exactly onto the image's outer pixel edges
          (fx / z = 64 makes the float32 projection exact): u = -0.5 and
          v = -0.5 fall in the first pixel, u = W - 0.5 and v = H - 0.5 out,
          each with a point on the nearest pixel's ray at the same depth;
      (d) a point at exactly tau from a lone vertex (not matched) and one a
          float nearer (matched)."""
    rng = np.random.default_rng(99)
    cam = dict(width=160, height=120, fx=131.25, fy=131.25, cx=79.5, cy=59.5)
    W, H = 160, 120
    V = 2000
    f32 = np.float32
    z = rng.uniform(0.6, 1.4, V)
    u = rng.uniform(-0.4, W - 0.6, V)
    vv = rng.uniform(-0.4, H - 0.6, V)
    v = np.stack([(u - cam["cx"]) * z / cam["fx"], (vv - cam["cy"]) * z / cam["fy"], z], 1).astype(np.float32)
    xyz = np.zeros((H, W, 3), np.float32)
    for i in rng.choice(1500, 4000):
        p = v[i] + rng.normal(0, 0.004, 3).astype(np.float32)
        pu = int(np.floor(cam["fx"] * p[0] / p[2] + cam["cx"] + 0.5))
        pv = int(np.floor(cam["fy"] * p[1] / p[2] + cam["cy"] + 0.5))
        if 0 <= pu < W and 16 <= pv < H:
            xyz[pv, pu] = _backproject(cam, pu, pv, p[2])
    # planted positions: rows 2 and 11, every ninth column from 4 to 139
    grid = [(4 + 9 * j, r) for r in (2, 11) for j in range(16)]
    where, pl = [], iter(grid)

    def put(pu, pv, p):
        xyz[pv, pu] = p
        where.append(pv * W + pu)

    ze = f32(2.05078125)
    for q in range(12):                                   # (a) copies
        pu, pv = next(pl)
        p = _backproject(cam, pu, pv, 2.5)
        v[q] = np.array([p[0], p[1], p[2] - f32(0.001)], np.float32)
        v[1500 + q] = v[q]
        put(pu, pv, p)
    dz = np.array([0.0, 0.0, 0.0078125], np.float32)      # (a) pairs around a point
    for q in range(14):
        pu, pv = next(pl)
        p = _backproject(cam, pu, pv, ze)
        v[1600 + 2 * q] = p + dz
        v[1601 + 2 * q] = p - dz
        put(pu, pv, p)
    below = float(np.nextafter(f32(1e-3), f32(0)))        # (b) near the camera
    for q, zv in enumerate((-0.05, 0.0, 1e-3, below)):
        pu, pv = 6 + 9 * q, 6
        p = _backproject(cam, pu, pv, 0.01)
        v[1700 + q] = np.array([p[0], p[1], zv], np.float32)
        put(pu, pv, p)
    v[1704] = np.array([(f32(-0.75) - f32(79.5)) / f32(64), (f32(100) - f32(59.5)) / f32(64), ze], np.float32)
    put(0, 100, _backproject(cam, 0, 100, ze))            # (b) u = -0.75: bucket -1
    for q, (eu, ev, pu, pv) in enumerate(((-0.5, 60.0, 0, 60), (W - 0.5, 60.0, W - 1, 60),  # (c)
                                          (155.0, -0.5, 155, 0), (155.0, H - 0.5, 155, H - 1))):
        v[1720 + q] = np.array([(f32(eu) - f32(79.5)) / f32(64), (f32(ev) - f32(59.5)) / f32(64), ze], np.float32)
        put(pu, pv, _backproject(cam, pu, pv, ze))
    for q, pd in enumerate((f32(2.125), np.nextafter(f32(2.125), f32(0)))):  # (d)
        pu, pv = next(pl)
        p = _backproject(cam, pu, pv, pd)
        v[1730 + q] = np.array([p[0], p[1], 2.0], np.float32)
        put(pu, pv, p)
    return cam, v, xyz, np.array(where)


def planted_expectations(cam, v32, xyz, where):
    """The oracle's association of the planted cloud, checked against brute
    force and against what each planted case is for."""
    a = oracle.associate(cam, 0.125, v32, xyz=xyz)
    np.testing.assert_array_equal(a, oracle.associate(cam, 0.125, v32, xyz=xyz, brute=True))
    assert (a >= 0).sum() > 1000
    pl = a[where]
    assert not np.isin(a, np.arange(1500, 1512)).any()                  # ties: the lower copy
    np.testing.assert_array_equal(pl[:12], np.arange(12))
    np.testing.assert_array_equal(pl[12:26], 1600 + 2 * np.arange(14))  # midway: the lower index
    assert not np.isin(a, np.arange(1700, 1705)).any() and (pl[26:31] == -1).all()
    np.testing.assert_array_equal(pl[31:35], [1720, -1, 1722, -1])     # pixel edges
    np.testing.assert_array_equal(pl[35:37], [-1, 1731])               # exactly tau, one float inside
    return a
