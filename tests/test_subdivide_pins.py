"""Pins of the template-refinement oracle (Section 3.3; Catmull and Clark's
rules): closed forms on a cube, counts, affine invariance, a planar grid,
and the skin weights carried by the same masks as the positions."""
import numpy as np

from oracle.subdivide import subdivide


def _cube():
    x = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                  [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], np.float64)
    quads = [[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]]
    fs = np.arange(0, 25, 4)
    return x, fs, np.array(quads).ravel()


def _one_link(V):
    return np.zeros((V, 1), np.int32), np.ones((V, 1))


def _edges(tris):
    e = set()
    for t in tris:
        for i in range(3):
            e.add(frozenset((int(t[i]), int(t[(i + 1) % 3]))))
    return e


def test_cube_first_round_closed_forms():
    x, fs, fv = _cube()
    P, tris, _, _ = subdivide(x, fs, fv, *_one_link(8), levels=1)
    assert P.shape == (8 + 12 + 6, 3) and tris.shape == (2 * 24, 3)
    # corner (valence 3): (Q + 2R)/3 with Q = -(1,1,1)/3, R = -2(1,1,1)/3 -> 5/9 of the corner
    np.testing.assert_allclose(P[:8], x * 5.0 / 9.0, atol=1e-15)
    # edge points: (two ends + two face centres) / 4 -> 3/4 off the edge's axis
    for q in range(8, 20):
        assert sorted(np.abs(P[q]).tolist()) == [0.0, 0.75, 0.75]
    # face points: the face centres
    for q in range(20, 26):
        assert sorted(np.abs(P[q]).tolist()) == [0.0, 0.0, 1.0]
    # closed surface after refinement: every edge in exactly two triangles,
    # Euler characteristic 2, every triangle facing outward
    E = _edges(tris)
    assert len(P) - len(E) + len(tris) == 2
    c = P[tris].mean(1)
    nrm = np.cross(P[tris[:, 1]] - P[tris[:, 0]], P[tris[:, 2]] - P[tris[:, 0]])
    assert (np.einsum("ij,ij->i", nrm, c) > 0).all()


def test_counts_after_two_rounds():
    x, fs, fv = _cube()
    P, tris, _, _ = subdivide(x, fs, fv, *_one_link(8), levels=2)
    # V1 = V + E + F = 26, E1 = 2E + sum deg = 48, F1 = 24; V2 = 26 + 48 + 24
    assert P.shape[0] == 98 and tris.shape[0] == 2 * 96


def test_affine_invariance():
    x, fs, fv = _cube()
    rng = np.random.default_rng(3)
    x = x + rng.normal(0, 0.2, x.shape)
    A = rng.normal(size=(3, 3))
    t = rng.normal(size=3)
    P, tris, _, _ = subdivide(x, fs, fv, *_one_link(8), levels=2)
    Q, tris2, _, _ = subdivide(x @ A.T + t, fs, fv, *_one_link(8), levels=2)
    np.testing.assert_allclose(Q, P @ A.T + t, atol=1e-12)


def _grid(n):
    x = np.array([[i, j, 0.0] for j in range(n) for i in range(n)], np.float64)
    quads = [[j * n + i, j * n + i + 1, (j + 1) * n + i + 1, (j + 1) * n + i]
             for j in range(n - 1) for i in range(n - 1)]
    fs = np.arange(0, 4 * len(quads) + 1, 4)
    return x, fs, np.array(quads).ravel()


def test_regular_planar_grid_refines_to_the_half_spacing_grid():
    """On a regular planar grid the rules are uniform cubic B-spline
    refinement: away from the boundary the new points are the grid at half
    the spacing, in the plane."""
    n = 7
    x, fs, fv = _grid(n)
    P, _, _, _ = subdivide(x, fs, fv, *_one_link(n * n), levels=1)
    assert np.abs(P[:, 2]).max() == 0.0
    inner = (P[:, 0] > 1.4) & (P[:, 0] < n - 2.4) & (P[:, 1] > 1.4) & (P[:, 1] < n - 2.4)
    assert inner.sum() > 10
    np.testing.assert_allclose(P[inner, :2] * 2, np.round(P[inner, :2] * 2), atol=1e-12)
    # the interior old vertices stay where they were (regular valence 4)
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            np.testing.assert_allclose(P[j * n + i], x[j * n + i], atol=1e-12)


def test_boundary_rules():
    n = 4
    x, fs, fv = _grid(n)
    P, _, _, _ = subdivide(x, fs, fv, *_one_link(n * n), levels=1)
    # a boundary vertex between two collinear boundary neighbours stays put
    np.testing.assert_allclose(P[1], x[1], atol=1e-15)
    # a corner (two boundary edges at a right angle): (a + b)/8 + 3/4 S
    np.testing.assert_allclose(P[0], (x[1] + x[n]) / 8 + 0.75 * x[0], atol=1e-15)


def test_weights_follow_the_position_masks():
    """Weights that are an affine function of the position (positive, two
    links) stay that function of the refined positions, and sum to one."""
    x, fs, fv = _cube()
    rng = np.random.default_rng(8)
    x = x + rng.normal(0, 0.1, x.shape)
    a, b = np.array([0.1, -0.05, 0.2]), 0.5
    w0 = x @ a + b
    assert ((w0 > 0) & (w0 < 1)).all()
    sl = np.tile([0, 1], (8, 1)).astype(np.int32)
    sw = np.stack([w0, 1 - w0], 1)
    P, _, L, W = subdivide(x, fs, fv, sl, sw, levels=2, max_infl_out=2)
    got0 = np.where(L == 0, W, 0).sum(1)
    np.testing.assert_allclose(got0, P @ a + b, atol=1e-12)
    np.testing.assert_allclose(W.sum(1), 1.0, atol=1e-12)


def test_weights_keep_the_largest_influences():
    x, fs, fv = _cube()
    sl = np.array([[q % 6, (q + 1) % 6, (q + 2) % 6] for q in range(8)], np.int32)
    sw = np.tile([0.5, 0.3, 0.2], (8, 1))
    P, _, L, W = subdivide(x, fs, fv, sl, sw, levels=1, max_infl_out=2)
    assert (L >= 0).all() and (np.diff(W, axis=1) <= 0).all()
    np.testing.assert_allclose(W.sum(1), 1.0, atol=1e-12)
