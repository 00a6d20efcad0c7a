"""Oracle of the template refinement (Section 3.3): Catmull-Clark
subdivision of a polygon mesh, skin weights carried with the same masks,
quadrilaterals split into triangles.  Test infrastructure: plain Python
loops in float64, small meshes only; written from Catmull and Clark's
rules, independently of the library.

The numbering of each round and the final split follow the library's
documented conventions (vertex points, then edge points in order of first
appearance, then face points; face f's corner i gives the quadrilateral
(v_i, e(v_i, v_i+1), f, e(v_i-1, v_i)); the shorter diagonal, ties through
the first corner), so that the two results compare index by index.
"""
import numpy as np


def _round(xyz, faces, weights):
    """One round.  xyz: list of 3-lists; faces: list of corner lists;
    weights: list of {link: weight}.  Returns the same for the next level."""
    nv = len(xyz)
    edge_of = {}          # frozenset({a, b}) -> edge number
    edge_ends = []
    edge_faces = []
    for f, corners in enumerate(faces):
        k = len(corners)
        for i in range(k):
            a, b = corners[i], corners[(i + 1) % k]
            key = frozenset((a, b))
            if key not in edge_of:
                edge_of[key] = len(edge_ends)
                edge_ends.append((a, b))
                edge_faces.append([])
            edge_faces[edge_of[key]].append(f)
    ne, nf = len(edge_ends), len(faces)

    def mix(terms):
        """sum of c * (position, weights) over (c, position, weights)"""
        p = [0.0, 0.0, 0.0]
        w = {}
        for c, q, wq in terms:
            for d in range(3):
                p[d] += c * q[d]
            for link, val in wq.items():
                w[link] = w.get(link, 0.0) + c * val
        return p, w

    fp = [mix([(1.0 / len(c), xyz[v], weights[v]) for v in c]) for c in faces]
    ep = []
    for e, (a, b) in enumerate(edge_ends):
        fs = edge_faces[e]
        if len(fs) == 1:
            ep.append(mix([(0.5, xyz[a], weights[a]), (0.5, xyz[b], weights[b])]))
        else:
            ep.append(mix([(0.25, xyz[a], weights[a]), (0.25, xyz[b], weights[b]),
                           (0.25, fp[fs[0]][0], fp[fs[0]][1]), (0.25, fp[fs[1]][0], fp[fs[1]][1])]))
    vp = [None] * nv
    inc_faces = [[] for _ in range(nv)]
    for f, c in enumerate(faces):
        for v in c:
            inc_faces[v].append(f)
    inc_edges = [[] for _ in range(nv)]
    for e, (a, b) in enumerate(edge_ends):
        inc_edges[a].append(e)
        inc_edges[b].append(e)
    for v in range(nv):
        es = inc_edges[v]
        border = [e for e in es if len(edge_faces[e]) == 1]
        if not es or (border and len(border) != 2):
            vp[v] = mix([(1.0, xyz[v], weights[v])])
        elif border:
            others = [edge_ends[e][0] if edge_ends[e][1] == v else edge_ends[e][1] for e in border]
            vp[v] = mix([(0.125, xyz[others[0]], weights[others[0]]), (0.125, xyz[others[1]], weights[others[1]]),
                         (0.75, xyz[v], weights[v])])
        else:
            n = float(len(es))
            terms = [(1.0 / (n * len(inc_faces[v])), fp[f][0], fp[f][1]) for f in inc_faces[v]]
            for e in es:
                a, b = edge_ends[e]
                # 2 R / n with R the mean of the edges' midpoints
                terms.append((1.0 / (n * n), xyz[a], weights[a]))
                terms.append((1.0 / (n * n), xyz[b], weights[b]))
            terms.append(((n - 3.0) / n, xyz[v], weights[v]))
            vp[v] = mix(terms)
    new_xyz = [p for p, _ in vp] + [p for p, _ in ep] + [p for p, _ in fp]
    new_w = [w for _, w in vp] + [w for _, w in ep] + [w for _, w in fp]
    new_faces = []
    for f, c in enumerate(faces):
        k = len(c)
        for i in range(k):
            e_next = edge_of[frozenset((c[i], c[(i + 1) % k]))]
            e_prev = edge_of[frozenset((c[(i - 1) % k], c[i]))]
            new_faces.append([c[i], nv + e_next, nv + ne + f, nv + e_prev])
    return new_xyz, new_faces, new_w


def subdivide(xyz, face_start, face_verts, skin_link, skin_w, levels=2, max_infl_out=4):
    """(xyz [V',3] float64, tris [T',3], skin_link [V',K], skin_w [V',K])."""
    pts = [list(map(float, p)) for p in np.asarray(xyz, np.float64)]
    fs = list(np.asarray(face_start, np.int64))
    fv = list(np.asarray(face_verts, np.int64))
    faces = [[int(v) for v in fv[fs[f]:fs[f + 1]]] for f in range(len(fs) - 1)]
    sl = np.asarray(skin_link)
    sw = np.asarray(skin_w, np.float64)
    weights = []
    for i in range(len(pts)):
        w = {}
        for k in range(sl.shape[1]):
            if sl[i, k] >= 0 and sw[i, k] != 0.0:
                w[int(sl[i, k])] = w.get(int(sl[i, k]), 0.0) + float(sw[i, k])
        weights.append(w)
    for _ in range(levels):
        pts, faces, weights = _round(pts, faces, weights)
    P = np.array(pts)
    tris = []
    for q in faces:
        a, b, c, d = q
        if np.sum((P[a] - P[c]) ** 2) <= np.sum((P[b] - P[d]) ** 2):
            tris += [[a, b, c], [a, c, d]]
        else:
            tris += [[a, b, d], [b, c, d]]
    K = max_infl_out
    out_l = np.full((len(pts), K), -1, np.int32)
    out_w = np.zeros((len(pts), K))
    for i, w in enumerate(weights):
        items = sorted([(l, v) for l, v in w.items() if v > 0.0], key=lambda t: (-t[1], t[0]))[:K]
        tot = sum(v for _, v in items)
        for k, (l, v) in enumerate(items):
            out_l[i, k] = l
            out_w[i, k] = v / tot
    return P, np.array(tris, np.int64), out_l, out_w
