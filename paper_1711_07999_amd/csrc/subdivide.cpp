// Template refinement (Section 3.3): a low-resolution polygon mesh with skin
// weights becomes the tracked high-resolution triangle mesh by rounds of
// Catmull-Clark subdivision, the weights carried through with the same
// averaging masks as the positions, the final quadrilaterals split into two
// triangles each.  Host code, run once per template.
//
// One round (Catmull and Clark 1978), for a mesh whose every edge has one
// or two faces:
//   face point    the mean of the face's vertices;
//   edge point    interior edge: the mean of its two ends and the two face
//                 points beside it; boundary edge: its midpoint;
//   vertex point  interior vertex of valence n: (Q + 2 R + (n - 3) S) / n,
//                 Q the mean of the face points around it, R the mean of the
//                 midpoints of its edges, S its position; a boundary vertex
//                 with two boundary edges to a and b: (a + b) / 8 + 3 S / 4;
//                 any other boundary vertex stays.
// Numbering of a round's output: the vertex points in input order, then the
// edge points in order of first appearance (faces in order, each face's
// edges from its first vertex on), then the face points in face order; face
// f with corners v_0 .. v_{k-1} gives the k quadrilaterals
// (v_i, e(v_i, v_i+1), f, e(v_i-1, v_i)), i = 0 .. k-1, in that order, which
// keeps the input's orientation.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/track.h"

int track_fail_message(int code, const char* msg);   // sets track_last_error (track.hip)

namespace {

// sparse weights of one vertex: (link, weight), links ascending
using Weights = std::vector<std::pair<int, double>>;

void axpy(Weights& acc, const Weights& w, double a) {
    for (const auto& lw : w) {
        auto it = std::lower_bound(acc.begin(), acc.end(), lw.first,
                                   [](const std::pair<int, double>& p, int l) { return p.first < l; });
        if (it != acc.end() && it->first == lw.first) it->second += a * lw.second;
        else acc.insert(it, {lw.first, a * lw.second});
    }
}

struct Mesh {
    std::vector<double> x;        // [V*3]
    std::vector<Weights> w;       // [V]
    std::vector<int> start, idx;  // polygon faces
    int nv() const { return (int)w.size(); }
    int nf() const { return (int)start.size() - 1; }
};

struct Edge { int a, b, f0, f1; };

int refine(const Mesh& in, Mesh& out, std::string& err) {
    const int V = in.nv(), F = in.nf();
    // edges in order of first appearance; a directed edge may occur once
    std::unordered_map<uint64_t, int> eid;
    std::unordered_map<uint64_t, int> directed;
    std::vector<Edge> edges;
    std::vector<int> face_edge(in.idx.size());   // edge of (corner i, corner i+1)
    for (int f = 0; f < F; ++f) {
        const int s = in.start[f], k = in.start[f + 1] - s;
        for (int i = 0; i < k; ++i) {
            const int a = in.idx[s + i], b = in.idx[s + (i + 1) % k];
            const uint64_t dk = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
            if (!directed.emplace(dk, f).second) {
                err = "edge " + std::to_string(a) + "-" + std::to_string(b) +
                      " is traversed twice in the same direction (inconsistent orientation or non-manifold)";
                return TRACK_E_INVALID;
            }
            const uint64_t key = ((uint64_t)(uint32_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
            auto it = eid.find(key);
            if (it == eid.end()) {
                eid.emplace(key, (int)edges.size());
                face_edge[s + i] = (int)edges.size();
                edges.push_back({a, b, f, -1});
            } else {
                Edge& e = edges[it->second];
                if (e.f1 >= 0) {
                    err = "edge " + std::to_string(a) + "-" + std::to_string(b) + " has more than two faces";
                    return TRACK_E_INVALID;
                }
                e.f1 = f;
                face_edge[s + i] = it->second;
            }
        }
    }
    const int E = (int)edges.size();
    const int NV = V + E + F;
    out.x.assign(3 * (size_t)NV, 0.0);
    out.w.assign(NV, Weights());
    // face points
    for (int f = 0; f < F; ++f) {
        const int s = in.start[f], k = in.start[f + 1] - s;
        double* p = &out.x[3 * (size_t)(V + E + f)];
        for (int i = 0; i < k; ++i) {
            const int v = in.idx[s + i];
            for (int d = 0; d < 3; ++d) p[d] += in.x[3 * (size_t)v + d] / k;
            axpy(out.w[V + E + f], in.w[v], 1.0 / k);
        }
    }
    // edge points
    for (int e = 0; e < E; ++e) {
        const Edge& g = edges[e];
        double* p = &out.x[3 * (size_t)(V + e)];
        Weights& w = out.w[V + e];
        if (g.f1 < 0) {
            for (int d = 0; d < 3; ++d) p[d] = 0.5 * (in.x[3 * (size_t)g.a + d] + in.x[3 * (size_t)g.b + d]);
            axpy(w, in.w[g.a], 0.5);
            axpy(w, in.w[g.b], 0.5);
        } else {
            const double* f0 = &out.x[3 * (size_t)(V + E + g.f0)];
            const double* f1 = &out.x[3 * (size_t)(V + E + g.f1)];
            for (int d = 0; d < 3; ++d)
                p[d] = 0.25 * (in.x[3 * (size_t)g.a + d] + in.x[3 * (size_t)g.b + d] + f0[d] + f1[d]);
            axpy(w, in.w[g.a], 0.25);
            axpy(w, in.w[g.b], 0.25);
            axpy(w, out.w[V + E + g.f0], 0.25);
            axpy(w, out.w[V + E + g.f1], 0.25);
        }
    }
    // vertex points: incident faces and edges of every vertex
    std::vector<std::vector<int>> vf(V), ve(V);
    for (int f = 0; f < F; ++f)
        for (int q = in.start[f]; q < in.start[f + 1]; ++q) vf[in.idx[q]].push_back(f);
    for (int e = 0; e < E; ++e) { ve[edges[e].a].push_back(e); ve[edges[e].b].push_back(e); }
    for (int v = 0; v < V; ++v) {
        double* p = &out.x[3 * (size_t)v];
        Weights& w = out.w[v];
        const double* S = &in.x[3 * (size_t)v];
        std::vector<int> bnd;
        for (int e : ve[v])
            if (edges[e].f1 < 0) bnd.push_back(e);
        if (ve[v].empty()) {   // unreferenced vertex: stays
            for (int d = 0; d < 3; ++d) p[d] = S[d];
            axpy(w, in.w[v], 1.0);
        } else if (!bnd.empty()) {
            if (bnd.size() == 2) {
                const int a = edges[bnd[0]].a == v ? edges[bnd[0]].b : edges[bnd[0]].a;
                const int b = edges[bnd[1]].a == v ? edges[bnd[1]].b : edges[bnd[1]].a;
                for (int d = 0; d < 3; ++d)
                    p[d] = 0.125 * (in.x[3 * (size_t)a + d] + in.x[3 * (size_t)b + d]) + 0.75 * S[d];
                axpy(w, in.w[a], 0.125);
                axpy(w, in.w[b], 0.125);
                axpy(w, in.w[v], 0.75);
            } else {
                for (int d = 0; d < 3; ++d) p[d] = S[d];
                axpy(w, in.w[v], 1.0);
            }
        } else {
            const double n = (double)ve[v].size();
            const double nfc = (double)vf[v].size();
            for (int d = 0; d < 3; ++d) {
                double Q = 0.0, R = 0.0;
                for (int f : vf[v]) Q += out.x[3 * (size_t)(V + E + f) + d];
                for (int e : ve[v]) R += 0.5 * (in.x[3 * (size_t)edges[e].a + d] + in.x[3 * (size_t)edges[e].b + d]);
                p[d] = (Q / nfc + 2.0 * R / n + (n - 3.0) * S[d]) / n;
            }
            for (int f : vf[v]) axpy(w, out.w[V + E + f], 1.0 / (nfc * n));
            for (int e : ve[v]) {
                axpy(w, in.w[edges[e].a], 1.0 / (n * n));
                axpy(w, in.w[edges[e].b], 1.0 / (n * n));
            }
            axpy(w, in.w[v], (n - 3.0) / n);
        }
    }
    // quadrilaterals
    out.start.assign(1, 0);
    out.idx.clear();
    for (int f = 0; f < F; ++f) {
        const int s = in.start[f], k = in.start[f + 1] - s;
        for (int i = 0; i < k; ++i) {
            out.idx.push_back(in.idx[s + i]);
            out.idx.push_back(V + face_edge[s + i]);
            out.idx.push_back(V + E + f);
            out.idx.push_back(V + face_edge[s + (i + k - 1) % k]);
            out.start.push_back((int)out.idx.size());
        }
    }
    return TRACK_OK;
}

double dist2(const std::vector<double>& x, int a, int b) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double t = x[3 * (size_t)a + d] - x[3 * (size_t)b + d];
        s += t * t;
    }
    return s;
}

}  // namespace

extern "C" int track_subdivide(const track_polymesh* in, int32_t levels, int32_t max_infl_out,
                               int32_t* n_verts_out, int32_t* n_tris_out, float* xyz_out, int32_t* tris_out,
                               int32_t* skin_link_out, float* skin_w_out) {
    if (!in || !n_verts_out || !n_tris_out) return track_fail_message(TRACK_E_INVALID, "mesh/size outputs are NULL");
    if (levels < 1 || levels > 4) return track_fail_message(TRACK_E_INVALID, "levels must be 1..4");
    if (max_infl_out < 1 || max_infl_out > TRACK_MAX_INFL)
        return track_fail_message(TRACK_E_INVALID, "max_infl_out must be 1..TRACK_MAX_INFL");
    if (in->n_verts < 3 || in->n_faces < 1 || !in->xyz || !in->face_start || !in->face_verts)
        return track_fail_message(TRACK_E_INVALID, "mesh needs vertices and faces");
    if (in->max_infl < 1 || !in->skin_link || !in->skin_w)
        return track_fail_message(TRACK_E_INVALID, "mesh needs skin weights");
    Mesh m;
    const int V = in->n_verts, F = in->n_faces, K = in->max_infl;
    m.x.resize(3 * (size_t)V);
    for (size_t q = 0; q < m.x.size(); ++q) m.x[q] = in->xyz[q];
    m.w.resize(V);
    for (int v = 0; v < V; ++v)
        for (int k = 0; k < K; ++k) {
            const int l = in->skin_link[(size_t)v * K + k];
            const float wt = in->skin_w[(size_t)v * K + k];
            if (l >= 0 && wt != 0.0f) axpy(m.w[v], Weights{{l, (double)wt}}, 1.0);
        }
    m.start.assign(in->face_start, in->face_start + F + 1);
    if (m.start[0] != 0) return track_fail_message(TRACK_E_INVALID, "face_start[0] must be 0");
    for (int f = 0; f < F; ++f)
        if (m.start[f + 1] - m.start[f] < 3) return track_fail_message(TRACK_E_INVALID, "a face has fewer than 3 corners");
    m.idx.assign(in->face_verts, in->face_verts + m.start[F]);
    for (int v : m.idx)
        if (v < 0 || v >= V) return track_fail_message(TRACK_E_INVALID, "face corner out of range");
    std::string err;
    for (int r = 0; r < levels; ++r) {
        Mesh next;
        const int rc = refine(m, next, err);
        if (rc) return track_fail_message(rc, err.c_str());
        m = std::move(next);
    }
    const long long nv = m.nv(), nt = 2LL * m.nf();
    if (nv > INT32_MAX / 3 || nt > INT32_MAX / 3) return track_fail_message(TRACK_E_INVALID, "refined mesh too large");
    *n_verts_out = (int32_t)nv;
    *n_tris_out = (int32_t)nt;
    if (xyz_out)
        for (size_t q = 0; q < m.x.size(); ++q) xyz_out[q] = (float)m.x[q];
    if (tris_out) {
        // every face is a quadrilateral after a round; split along the
        // shorter diagonal (ties: the one through the first corner)
        for (int f = 0; f < m.nf(); ++f) {
            const int* q = &m.idx[m.start[f]];
            int32_t* t = tris_out + 6 * (size_t)f;
            if (dist2(m.x, q[0], q[2]) <= dist2(m.x, q[1], q[3])) {
                t[0] = q[0]; t[1] = q[1]; t[2] = q[2]; t[3] = q[0]; t[4] = q[2]; t[5] = q[3];
            } else {
                t[0] = q[0]; t[1] = q[1]; t[2] = q[3]; t[3] = q[1]; t[4] = q[2]; t[5] = q[3];
            }
        }
    }
    if (skin_link_out || skin_w_out) {
        // the largest max_infl_out weights of each vertex (ties: the lower
        // link), scaled to sum to one
        for (int v = 0; v < m.nv(); ++v) {
            Weights w = m.w[v];
            w.erase(std::remove_if(w.begin(), w.end(), [](const std::pair<int, double>& p) { return !(p.second > 0.0); }),
                    w.end());
            std::stable_sort(w.begin(), w.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
                return a.second > b.second || (a.second == b.second && a.first < b.first);
            });
            if ((int)w.size() > max_infl_out) w.resize(max_infl_out);
            double tot = 0.0;
            for (const auto& p : w) tot += p.second;
            for (int k = 0; k < max_infl_out; ++k) {
                const bool has = k < (int)w.size() && tot > 0.0;
                if (skin_link_out) skin_link_out[(size_t)v * max_infl_out + k] = has ? w[k].first : -1;
                if (skin_w_out) skin_w_out[(size_t)v * max_infl_out + k] = has ? (float)(w[k].second / tot) : 0.0f;
            }
        }
    }
    return TRACK_OK;
}
