"""Tracking-quality measures of the paper's experiments (Section 5), computed
on the host from tracked states: joint-position accuracy as a function of
the distance threshold (Section 5.1 plots accuracy against the threshold
instead of fixing one), the area under that curve, and the reconstruction
error of the visible surface (Section 5.3: distance from each visible model
vertex to the nearest observed point of the frame).

Tracking modes of Section 5.1, as per-frame schedules of the same step
(see `mode_schedule`): the full method (pose and offsets on every
iteration), shape match (offsets estimated on the first frame only, then
held), smooth bind (pose only, offsets zero), rigid segments (pose only on
a model whose vertices each follow one link), and the paper's per-frame
iteration counts (Section 4.2: ten to fifteen pose iterations; Section 4.3:
two offset iterations after them), also with the linear variant of the
blend (see `model_for`).
"""
import numpy as np

MODES = ("full", "shape-match", "smooth-bind", "rigid-segments", "paper-schedule", "paper-schedule-linear")


def mode_schedule(mode: str, frame: int, n_iters: int):
    """(do_pose, do_shape) uint8 flag arrays of `frame` (0-based) in `mode`;
    `n_iters` is the iteration count of the full method."""
    one = np.ones(n_iters, np.uint8)
    zero = np.zeros(n_iters, np.uint8)
    if mode == "full":
        return one, one.copy()
    if mode == "shape-match":
        return one, (one.copy() if frame == 0 else zero)
    if mode in ("smooth-bind", "rigid-segments"):
        return one, zero
    if mode in ("paper-schedule", "paper-schedule-linear"):
        p = np.array([1] * 12 + [0] * 2, np.uint8)
        return p, 1 - p
    raise ValueError(f"unknown mode {mode!r}")


def model_for(mode: str, model: dict) -> dict:
    """The template a mode tracks with."""
    if mode == "rigid-segments":
        return rigid_segments(model)
    if mode == "paper-schedule-linear":
        return dict(model, blend=1)
    return model


def rigid_segments(model: dict) -> dict:
    """The model with every vertex following only its largest-weight link
    (ties to the lower slot): a mesh of rigid segments, one per link."""
    m = dict(model)
    w = np.asarray(model["skin_w"], np.float32)
    links = np.asarray(model["skin_link"], np.int32)
    k = np.argmax(np.where(links >= 0, w, -1.0), axis=1)
    rows = np.arange(w.shape[0])
    sl = np.full_like(links, -1)
    sw = np.zeros_like(w)
    sl[rows, 0] = links[rows, k]
    sw[rows, 0] = 1.0
    m["skin_link"], m["skin_w"] = sl, sw
    return m


def joint_errors(pred: np.ndarray, true: np.ndarray) -> np.ndarray:
    """Euclidean distance per joint (last axis = xyz)."""
    return np.linalg.norm(np.asarray(pred, np.float64) - np.asarray(true, np.float64), axis=-1)


def accuracy_curve(errors: np.ndarray, thresholds: np.ndarray) -> np.ndarray:
    """Fraction of joint estimates within each distance threshold."""
    e = np.sort(np.asarray(errors, np.float64).ravel())
    return np.searchsorted(e, np.asarray(thresholds, np.float64), side="right") / max(e.size, 1)


def curve_auc(thresholds: np.ndarray, fractions: np.ndarray) -> float:
    """Area under an accuracy curve, normalised by the threshold range (1 =
    every joint exact), trapezoidal rule."""
    t = np.asarray(thresholds, np.float64)
    f = np.asarray(fractions, np.float64)
    return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(t)) / (t[-1] - t[0]))


def visible_vertices(verts: np.ndarray, normals: np.ndarray, cam: dict, tol: float = 0.01,
                     gap: float = 0.05, splat: int = 1) -> np.ndarray:
    """Vertices seen by the camera: in front of it, projecting into the
    image, facing it (normal against the viewing ray), within `tol` of the
    nearest facing vertex in their own pixel, and within `gap` of the
    nearest one over the (2 splat + 1)^2 pixels around it.  The second test
    closes the holes between the projections of neighbouring vertices (a
    hidden vertex seen through such a hole lies far behind the surface
    around it, while a slanted visible surface changes by less than `gap`
    from pixel to pixel)."""
    v = np.asarray(verts, np.float64)
    n = np.asarray(normals, np.float64)
    W, H = int(cam["width"]), int(cam["height"])
    z = v[:, 2]
    ok = z > 1e-3
    zs = np.where(ok, z, 1.0)
    u = np.floor(cam["fx"] * v[:, 0] / zs + cam["cx"] + 0.5).astype(np.int64)
    r = np.floor(cam["fy"] * v[:, 1] / zs + cam["cy"] + 0.5).astype(np.int64)
    ok &= (u >= 0) & (u < W) & (r >= 0) & (r < H)
    ok &= np.einsum("ij,ij->i", n, v) < 0.0
    pix = np.where(ok, r * W + u, 0)
    zown = np.full(W * H, np.inf)
    np.minimum.at(zown, pix[ok], z[ok])
    znb = np.full(W * H, np.inf)
    for du in range(-splat, splat + 1):
        for dv in range(-splat, splat + 1):
            uu, rr = u + du, r + dv
            inside = ok & (uu >= 0) & (uu < W) & (rr >= 0) & (rr < H)
            np.minimum.at(znb, (rr * W + uu)[inside], z[inside])
    return ok & (z <= zown[pix] + tol) & (z <= znb[pix] + gap)


def observed_points(depth: np.ndarray, cam: dict) -> np.ndarray:
    """Back-projected valid pixels of a depth image, [n, 3] float64."""
    d = np.asarray(depth, np.float64)
    H, W = d.shape
    vv, uu = np.nonzero(np.isfinite(d) & (d > 0))
    z = d[vv, uu]
    return np.stack([(uu - cam["cx"]) * z / cam["fx"], (vv - cam["cy"]) * z / cam["fy"], z], 1)


def reconstruction_errors(verts: np.ndarray, normals: np.ndarray, depth: np.ndarray, cam: dict) -> np.ndarray:
    """Distance from every visible vertex to the nearest observed point."""
    from scipy.spatial import cKDTree

    vis = visible_vertices(verts, normals, cam)
    pts = observed_points(depth, cam)
    if not vis.any() or pts.shape[0] == 0:
        return np.zeros(0)
    d, _ = cKDTree(pts).query(np.asarray(verts, np.float64)[vis])
    return d


def vertex_normals(verts: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """Area-weighted vertex normals of a triangle mesh (for visibility)."""
    v = np.asarray(verts, np.float64)
    f = np.asarray(faces, np.int64)
    c = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    n = np.zeros_like(v)
    for k in range(3):
        np.add.at(n, f[:, k], c)
    ln = np.linalg.norm(n, axis=1, keepdims=True)
    return n / np.where(ln > 0, ln, 1.0)
