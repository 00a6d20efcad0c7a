// Plain CPU oracle of the per-frame Gauss-Newton tracking step of
// "Dynamic High Resolution Deformable Articulated Tracking" (Walsman, Wan,
// Schmidt, Fox; 3DV 2017).
//
// TEST INFRASTRUCTURE.  This code exists to check the GPU library; only the
// test suite, the smoke check and the CPU-baseline leg of the benchmark load
// it.  It shares no source, header or table with the GPU library.
//
// Every function is a slow, direct transcription of the paper's definitions:
// loops over joints, vertices and pixels in index order, no blocking, no
// fusion.  The scalar type S is double for the reference runs and a forward
// dual number for the derivative pins (`real`, the scalar of the rest, is
// double too; only the CPU timing baseline builds a float instantiation).  Where the paper is silent or garbled
// the reading used is stated at the function (the same readings are listed
// in the design notes of the repository).
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#include <algorithm>

#ifndef ORC_REAL
#define ORC_REAL double   // the scalar of the reference runs
#define ORC_NS orc
#endif

namespace ORC_NS {

// Scalar of the oracle's arithmetic: double for every reference run and pin;
// a second instantiation in float (namespace orc32) serves only as a timing
// baseline at the GPU path's precision.
using real = ORC_REAL;

// ---------------------------------------------------------------------------
// forward dual number (value + one directional derivative), for pins only
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
    Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sin(Dual a) { return {std::sin(a.v), a.d * std::cos(a.v)}; }
inline Dual cos(Dual a) { return {std::cos(a.v), -a.d * std::sin(a.v)}; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, a.d / (2.0 * s)}; }
template <class T> inline T val(T a) { return a; }
inline double val(Dual a) { return a.v; }
using std::sin; using std::cos; using std::sqrt;

// ---------------------------------------------------------------------------
// quaternions and dual quaternions (Section 3.1)
// ---------------------------------------------------------------------------
template <class S> struct Quat { S w, x, y, z; };

template <class S> Quat<S> qmul(const Quat<S>& a, const Quat<S>& b) {
    return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
            a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
            a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
template <class S> Quat<S> qconj(const Quat<S>& a) { return {a.w, -a.x, -a.y, -a.z}; }
template <class S> Quat<S> qadd(const Quat<S>& a, const Quat<S>& b) {
    return {a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class S> Quat<S> qscale(const Quat<S>& a, S s) { return {a.w * s, a.x * s, a.y * s, a.z * s}; }
template <class S> S qdot(const Quat<S>& a, const Quat<S>& b) {
    return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}

// H = q_r + eps q_d with eps^2 = 0.
template <class S> struct DQ { Quat<S> r, d; };

template <class S> DQ<S> dq_identity() { return {{S(1), S(0), S(0), S(0)}, {S(0), S(0), S(0), S(0)}}; }
template <class S> DQ<S> dq_mul(const DQ<S>& a, const DQ<S>& b) {
    return {qmul(a.r, b.r), qadd(qmul(a.r, b.d), qmul(a.d, b.r))};
}
// inverse of a unit dual quaternion: conjugate both parts
template <class S> DQ<S> dq_inv_unit(const DQ<S>& a) { return {qconj(a.r), qconj(a.d)}; }
template <class S> DQ<S> dq_add(const DQ<S>& a, const DQ<S>& b) { return {qadd(a.r, b.r), qadd(a.d, b.d)}; }
template <class S> DQ<S> dq_scale(const DQ<S>& a, S s) { return {qscale(a.r, s), qscale(a.d, s)}; }

// Eq. (1): hinge, rotation by theta about unit axis z.
template <class S> DQ<S> dq_hinge(S th, const real z[3]) {
    S c = cos(th * S(0.5)), s = sin(th * S(0.5));
    return {{c, s * S(z[0]), s * S(z[1]), s * S(z[2])}, {S(0), S(0), S(0), S(0)}};
}
// Eq. (2): prismatic, translation by theta along unit axis z.
template <class S> DQ<S> dq_prismatic(S th, const real z[3]) {
    S h = th * S(0.5);
    return {{S(1), S(0), S(0), S(0)}, {S(0), h * S(z[0]), h * S(z[1]), h * S(z[2])}};
}
// Derivatives of Eq. (1) and (2) with respect to theta (Section 4.2).
template <class S> DQ<S> dq_hinge_dtheta(S th, const real z[3]) {
    S c = cos(th * S(0.5)) * S(0.5), s = sin(th * S(0.5)) * S(0.5);
    return {{-s, c * S(z[0]), c * S(z[1]), c * S(z[2])}, {S(0), S(0), S(0), S(0)}};
}
template <class S> DQ<S> dq_prismatic_dtheta(const real z[3]) {
    return {{S(0), S(0), S(0), S(0)}, {S(0), S(real(0.5) * z[0]), S(real(0.5) * z[1]), S(real(0.5) * z[2])}};
}
// Rigid transform x -> R(q) x + t as a dual quaternion: (q, 1/2 t q).
template <class S> DQ<S> dq_from_rt(const real q[4], const real t[3]) {
    Quat<S> r{S(q[0]), S(q[1]), S(q[2]), S(q[3])};
    Quat<S> tq{S(0), S(real(0.5) * t[0]), S(real(0.5) * t[1]), S(real(0.5) * t[2])};
    return {r, qmul(tq, r)};
}

// Point transform by a (possibly blended, non-unit) dual quaternion
// H = (r, d):  T(H, x) = (r x conj(r) + 2 vec(d conj(r))) / (r . r).
// For a unit H this is the rigid motion H encodes; for a blend it equals the
// normalised dual-quaternion blend of Kavan et al. that Section 3.2 cites.
template <class S> void dq_transform(const DQ<S>& H, const S x[3], S out[3]) {
    Quat<S> xq{S(0), x[0], x[1], x[2]};
    Quat<S> a = qmul(qmul(H.r, xq), qconj(H.r));
    Quat<S> b = qmul(H.d, qconj(H.r));
    S nn = qdot(H.r, H.r);
    out[0] = (a.x + S(2) * b.x) / nn;
    out[1] = (a.y + S(2) * b.y) / nn;
    out[2] = (a.z + S(2) * b.z) / nn;
}

// Rotation matrix of r / |r| (row-major), which is dT/dx.
template <class S> void quat_rotation(const Quat<S>& r, S R[9]) {
    S n = qdot(r, r);
    S w = r.w, x = r.x, y = r.y, z = r.z;
    S s = S(2) / n;
    R[0] = S(1) - s * (y * y + z * z); R[1] = s * (x * y - w * z); R[2] = s * (x * z + w * y);
    R[3] = s * (x * y + w * z); R[4] = S(1) - s * (x * x + z * z); R[5] = s * (y * z - w * x);
    R[6] = s * (x * z - w * y); R[7] = s * (y * z + w * x); R[8] = S(1) - s * (x * x + y * y);
}

// dT/dH as a 3x8 matrix (columns r.w r.x r.y r.z d.w d.x d.y d.z), obtained
// by differentiating T(H, x) above term by term.
template <class S> void dq_transform_jacobian(const DQ<S>& H, const S x[3], S Jt[3][8]) {
    S T[3];
    dq_transform(H, x, T);
    S nn = qdot(H.r, H.r);
    Quat<S> xq{S(0), x[0], x[1], x[2]};
    const Quat<S> basis[4] = {{S(1), S(0), S(0), S(0)}, {S(0), S(1), S(0), S(0)},
                              {S(0), S(0), S(1), S(0)}, {S(0), S(0), S(0), S(1)}};
    Quat<S> rc = qconj(H.r);
    for (int c = 0; c < 4; ++c) {
        const Quat<S>& e = basis[c];
        // d/d r_c of numerator: e x r* + r x e* + 2 d e*
        Quat<S> t1 = qmul(qmul(e, xq), rc);
        Quat<S> t2 = qmul(qmul(H.r, xq), qconj(e));
        Quat<S> t3 = qmul(H.d, qconj(e));
        // d/d r_c of 1/nn = -2 r_c / nn^2
        S rcomp = (c == 0) ? H.r.w : (c == 1) ? H.r.x : (c == 2) ? H.r.y : H.r.z;
        Jt[0][c] = (t1.x + t2.x + S(2) * t3.x) / nn - T[0] * S(2) * rcomp / nn;
        Jt[1][c] = (t1.y + t2.y + S(2) * t3.y) / nn - T[1] * S(2) * rcomp / nn;
        Jt[2][c] = (t1.z + t2.z + S(2) * t3.z) / nn - T[2] * S(2) * rcomp / nn;
        // d/d d_c: 2 e r* / nn
        Quat<S> t4 = qmul(e, rc);
        Jt[0][4 + c] = S(2) * t4.x / nn;
        Jt[1][4 + c] = S(2) * t4.y / nn;
        Jt[2][4 + c] = S(2) * t4.z / nn;
    }
}

// ---------------------------------------------------------------------------
// inputs
// ---------------------------------------------------------------------------
enum { HINGE = 0, PRISMATIC = 1 };

enum { BLEND_DQ = 0, BLEND_LINEAR = 1 };

struct Model {
    int P = 0, L = 0, V = 0, F = 0, K = 0;
    int blend = BLEND_DQ;   // how a vertex's links are combined (see skin)
    std::vector<int> parent, type, link_joint, faces, skin_link, nbr;
    std::vector<real> axis, offq, offt, rest, skin_w;
    // derived
    std::vector<std::vector<char>> anc;  // anc[l][k]: joint k on the chain of link l
};

struct Camera { int W, H; float fx, fy, cx, cy; };

struct Params {
    float tau = 0.05f;
    int n_iters = 1;
    std::vector<uint8_t> do_pose, do_shape, active;
    real lambda_k = 0.01, lambda_s = 0.0, lambda_phi = 0.01, lambda_nbr = 1.0,
           lambda_t = 0.0, lambda_w = 0.1;
};

inline void model_derive(Model& m) {
    m.anc.assign(m.L, std::vector<char>(m.P, 0));
    for (int l = 0; l < m.L; ++l)
        for (int k = m.link_joint[l]; k >= 0; k = m.parent[k]) m.anc[l][k] = 1;
}

// ---------------------------------------------------------------------------
// Section 3.1: forward kinematics H_{0,j} = H_{0,P(j)} H_{P(j),j} H_j
// ---------------------------------------------------------------------------
template <class S> std::vector<DQ<S>> forward_kinematics(const Model& m, const S* theta) {
    std::vector<DQ<S>> H(m.P);
    for (int j = 0; j < m.P; ++j) {
        DQ<S> base = m.parent[j] < 0 ? dq_identity<S>() : H[m.parent[j]];
        DQ<S> off = dq_from_rt<S>(&m.offq[4 * j], &m.offt[3 * j]);
        DQ<S> Hj = m.type[j] == HINGE ? dq_hinge<S>(theta[j], &m.axis[3 * j])
                                      : dq_prismatic<S>(theta[j], &m.axis[3 * j]);
        H[j] = dq_mul(dq_mul(base, off), Hj);
    }
    return H;
}

// Section 3.2 / 4.2: link offsets H_{l,Delta} = H_{0,l} (H^0_{0,l})^{-1},
// with the bind pose H^0 at Theta = 0.
template <class S> std::vector<DQ<S>> link_deltas(const Model& m, const std::vector<DQ<S>>& H,
                                                 const std::vector<DQ<S>>& H0) {
    std::vector<DQ<S>> D(m.L);
    for (int l = 0; l < m.L; ++l) {
        int j = m.link_joint[l];
        D[l] = dq_mul(H[j], dq_inv_unit(H0[j]));
    }
    return D;
}

template <class S> std::vector<DQ<S>> bind_pose(const Model& m) {
    std::vector<S> z(m.P, S(0));
    return forward_kinematics<S>(m, z.data());
}

// Sign of each influence relative to the largest-weight influence (ties: the
// lower link index), so the blend stays on one hemisphere of the quaternion
// real cover.  The paper does not state this; it is Kavan et al.'s rule for
// dual-quaternion blending.
template <class S> void blend_signs(const Model& m, const std::vector<DQ<S>>& D, int i, S sgn[4]) {
    int piv = -1;
    real wbest = -1.0;
    for (int k = 0; k < m.K; ++k) {
        int l = m.skin_link[i * m.K + k];
        real w = m.skin_w[i * m.K + k];
        if (l < 0) continue;
        if (w > wbest || (w == wbest && l < m.skin_link[i * m.K + piv])) { wbest = w; piv = k; }
    }
    for (int k = 0; k < m.K; ++k) {
        int l = m.skin_link[i * m.K + k];
        sgn[k] = S(1);
        if (l < 0 || piv < 0) continue;
        S d = qdot(D[l].r, D[m.skin_link[i * m.K + piv]].r);
        if (val(d) < real(0)) sgn[k] = S(-1);
    }
}

// Eq. (3): blended dual quaternion H_{i,Sigma} = sum_j w_ij H_{j,Delta}.
template <class S> DQ<S> blend(const Model& m, const std::vector<DQ<S>>& D, int i) {
    S sgn[4];
    blend_signs(m, D, i, sgn);
    DQ<S> acc{{S(0), S(0), S(0), S(0)}, {S(0), S(0), S(0), S(0)}};
    for (int k = 0; k < m.K; ++k) {
        int l = m.skin_link[i * m.K + k];
        if (l < 0) continue;
        acc = dq_add(acc, dq_scale(D[l], S(m.skin_w[i * m.K + k]) * sgn[k]));
    }
    return acc;
}

// Eq. (5): v_i = H_{i,Sigma} (v0_i + phi_i).  The linear variant (matrix
// linear blend skinning) instead transforms the point rigidly by each link and
// averages the results with the weights: v_i = sum_j w_ij T(H_{j,Delta}, x_i).
template <class S> void skin(const Model& m, const std::vector<DQ<S>>& D, const S* phi, S* v) {
    for (int i = 0; i < m.V; ++i) {
        S x[3] = {S(m.rest[3 * i]) + phi[3 * i], S(m.rest[3 * i + 1]) + phi[3 * i + 1],
                  S(m.rest[3 * i + 2]) + phi[3 * i + 2]};
        if (m.blend == BLEND_LINEAR) {
            S acc[3] = {S(0), S(0), S(0)};
            for (int k = 0; k < m.K; ++k) {
                int l = m.skin_link[i * m.K + k];
                if (l < 0) continue;
                S y[3];
                dq_transform(D[l], x, y);
                for (int d = 0; d < 3; ++d) acc[d] = acc[d] + S(m.skin_w[i * m.K + k]) * y[d];
            }
            for (int d = 0; d < 3; ++d) v[3 * i + d] = acc[d];
        } else {
            DQ<S> H = blend(m, D, i);
            dq_transform(H, x, &v[3 * i]);
        }
    }
}

// d v_i / d x_i: the rotation of the blend (dual quaternions), or the
// weighted sum of the links' rotations (linear variant).
inline void point_jacobian(const Model& m, const std::vector<DQ<real>>& D, int i, real R[9]) {
    if (m.blend == BLEND_LINEAR) {
        std::fill(R, R + 9, 0.0);
        for (int k = 0; k < m.K; ++k) {
            int l = m.skin_link[i * m.K + k];
            if (l < 0) continue;
            real Rl[9];
            quat_rotation(D[l].r, Rl);
            for (int q = 0; q < 9; ++q) R[q] += m.skin_w[i * m.K + k] * Rl[q];
        }
    } else {
        quat_rotation(blend(m, D, i).r, R);
    }
}

// Vertex normals of the skinned mesh (Section 4.1 takes the residual along
// the vertex normal without defining it): sum over incident faces (a,b,c), in
// face order, of (v_b - v_a) x (v_c - v_a) -- each face weighted by twice its
// area -- normalised; zero if the sum is zero.
inline void vertex_normals(const Model& m, const real* v, real* n) {
    std::fill(n, n + 3 * m.V, 0.0);
    for (int f = 0; f < m.F; ++f) {
        int a = m.faces[3 * f], b = m.faces[3 * f + 1], c = m.faces[3 * f + 2];
        real e1[3], e2[3];
        for (int d = 0; d < 3; ++d) { e1[d] = v[3 * b + d] - v[3 * a + d]; e2[d] = v[3 * c + d] - v[3 * a + d]; }
        real cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        for (int d = 0; d < 3; ++d) { n[3 * a + d] += cr[d]; n[3 * b + d] += cr[d]; n[3 * c + d] += cr[d]; }
    }
    for (int i = 0; i < m.V; ++i) {
        real l = std::sqrt(n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2]);
        for (int d = 0; d < 3; ++d) n[3 * i + d] = l > real(0) ? n[3 * i + d] / l : real(0);
    }
}

// ---------------------------------------------------------------------------
// Section 4.1: observation points and projective association
// ---------------------------------------------------------------------------
// All association decisions are taken in float32 with this fixed operation
// order, built without floating-point contraction (-ffp-contract=off, no
// fused multiply-add): back-projection x = ((u - cx) * d) / fx,
// projection floor((fx * x) / z + cx + 0.5), squared distance
// (dx*dx + dy*dy) + dz*dz, acceptance d2 < tau*tau, ties to the lower index.
constexpr float kZNear = 1e-3f;

inline bool point_of_pixel(const Camera& c, const float* depth, const float* xyz, int k, float p[3]) {
    if (xyz) {
        p[0] = xyz[3 * k]; p[1] = xyz[3 * k + 1]; p[2] = xyz[3 * k + 2];
        return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]) && p[2] > 0.0f;
    }
    float d = depth[k];
    if (!(d > 0.0f) || !std::isfinite(d)) return false;
    int u = k % c.W, v = k / c.W;
    p[0] = (((float)u - c.cx) * d) / c.fx;
    p[1] = (((float)v - c.cy) * d) / c.fy;
    p[2] = d;
    return true;
}

// Vertex i is a candidate if it lies in front of the camera and projects into
// the image; its bucket is the rounded pixel.
inline bool vertex_pixel(const Camera& c, const float v[3], int* iu, int* iv) {
    if (!(v[2] > kZNear)) return false;
    float fu = std::floor((c.fx * v[0]) / v[2] + c.cx + 0.5f);
    float fv = std::floor((c.fy * v[1]) / v[2] + c.cy + 0.5f);
    if (!(fu >= 0.0f && fu < (float)c.W && fv >= 0.0f && fv < (float)c.H)) return false;
    *iu = (int)fu; *iv = (int)fv;
    return true;
}

inline float dist2(const float a[3], const float b[3]) {
    float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

// a(k) = argmin over candidate vertices with d2 < tau^2 (ties: lower index),
// -1 if none.  Brute force over all candidates.
inline void associate_brute(const Camera& c, float tau, const float* v, int V, const float* depth,
                            const float* xyz, int32_t* a) {
    const float t2 = tau * tau;
    std::vector<char> cand(V);
    for (int i = 0; i < V; ++i) { int u, w; cand[i] = vertex_pixel(c, &v[3 * i], &u, &w); }
    for (int k = 0; k < c.W * c.H; ++k) {
        a[k] = -1;
        float p[3];
        if (!point_of_pixel(c, depth, xyz, k, p)) continue;
        float best = t2;
        for (int i = 0; i < V; ++i) {
            if (!cand[i]) continue;
            float d2 = dist2(&v[3 * i], p);
            if (d2 < t2 && (a[k] < 0 || d2 < best)) { best = d2; a[k] = i; }
        }
    }
}

// Same result through a uniform 3-D grid of cell size slightly above tau:
// every vertex closer than tau lies in one of the 27 cells around the point.
inline void associate_grid(const Camera& c, float tau, const float* v, int V, const float* depth,
                           const float* xyz, int32_t* a) {
    const float t2 = tau * tau;
    real cell = (real)tau * real(1.001);
    struct Item { int64_t key; int i; };
    std::vector<Item> items;
    auto cellof = [&](real x) { return (int64_t)std::floor(x / cell); };
    auto keyof = [](int64_t x, int64_t y, int64_t z) {
        return ((x + (1 << 20)) << 42) | ((y + (1 << 20)) << 21) | (z + (1 << 20));
    };
    for (int i = 0; i < V; ++i) {
        int u, w;
        if (!vertex_pixel(c, &v[3 * i], &u, &w)) continue;
        items.push_back({keyof(cellof(v[3 * i]), cellof(v[3 * i + 1]), cellof(v[3 * i + 2])), i});
    }
    std::sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
        return x.key < y.key || (x.key == y.key && x.i < y.i);
    });
    std::vector<int64_t> keys(items.size());
    for (size_t q = 0; q < items.size(); ++q) keys[q] = items[q].key;
#pragma omp parallel for schedule(dynamic, 256)
    for (int k = 0; k < c.W * c.H; ++k) {
        a[k] = -1;
        float p[3];
        if (!point_of_pixel(c, depth, xyz, k, p)) continue;
        int64_t cx = cellof(p[0]), cy = cellof(p[1]), cz = cellof(p[2]);
        float best = t2;
        int bi = -1;
        for (int64_t dx = -1; dx <= 1; ++dx)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dz = -1; dz <= 1; ++dz) {
                    int64_t key = keyof(cx + dx, cy + dy, cz + dz);
                    auto it = std::lower_bound(keys.begin(), keys.end(), key);
                    for (size_t q = it - keys.begin(); q < keys.size() && keys[q] == key; ++q) {
                        int i = items[q].i;
                        float d2 = dist2(&v[3 * i], p);
                        if (d2 < t2 && (bi < 0 || d2 < best || (d2 == best && i < bi))) { best = d2; bi = i; }
                    }
                }
        a[k] = bi;
    }
}

// Section 4.1 (averaging): c_i = number of points whose closest vertex is i,
// delta_i = (1/c_i) sum_k (p_k - v_i), summed in ascending pixel order.
inline void average_offsets(const Camera& c, const float* depth, const float* xyz, const int32_t* a,
                            const real* v, int V, int32_t* cnt, real* delta) {
    std::fill(cnt, cnt + V, 0);
    std::fill(delta, delta + 3 * V, 0.0);
    for (int k = 0; k < c.W * c.H; ++k) {
        int i = a[k];
        if (i < 0) continue;
        float p[3];
        point_of_pixel(c, depth, xyz, k, p);
        cnt[i] += 1;
        for (int d = 0; d < 3; ++d) delta[3 * i + d] += (real)p[d] - v[3 * i + d];
    }
    for (int i = 0; i < V; ++i)
        if (cnt[i] > 0)
            for (int d = 0; d < 3; ++d) delta[3 * i + d] /= (real)cnt[i];
}

// ---------------------------------------------------------------------------
// Section 4.2: residuals, pose Jacobian, normal equations, damped step
// ---------------------------------------------------------------------------
// Block of dH_{l,Delta}/dtheta_k for joint k on the chain of link l:
//   H_{0,P(k)} H_{P(k),k} (dH_k/dtheta_k) H_{k,l} (H^0_{0,l})^{-1}
// with H_{k,l} = H_{0,k}^{-1} H_{0,l}.  (The printed block ends in H_{j,Delta};
// the trailing factor must be the inverse bind pose for the product to be the
// derivative of H_{0,l} (H^0_{0,l})^{-1}.)
inline DQ<real> delta_derivative(const Model& m, const std::vector<DQ<real>>& H,
                                   const std::vector<DQ<real>>& H0, const real* theta, int k, int l) {
    int jl = m.link_joint[l];
    DQ<real> base = m.parent[k] < 0 ? dq_identity<real>() : H[m.parent[k]];
    DQ<real> off = dq_from_rt<real>(&m.offq[4 * k], &m.offt[3 * k]);
    DQ<real> dHk = m.type[k] == HINGE ? dq_hinge_dtheta<real>(theta[k], &m.axis[3 * k])
                                        : dq_prismatic_dtheta<real>(&m.axis[3 * k]);
    DQ<real> Hkl = dq_mul(dq_inv_unit(H[k]), H[jl]);
    return dq_mul(dq_mul(dq_mul(dq_mul(base, off), dHk), Hkl), dq_inv_unit(H0[jl]));
}

struct PoseSystem {
    std::vector<real> J;   // [V*P], zero rows for vertices outside O
    std::vector<real> r;   // [V]
    std::vector<char> obs;   // [V] membership of O
    std::vector<real> A;   // [P*P] J^T J (+ prior)
    std::vector<real> b;   // [P]   J^T r (+ prior)
    real rr = 0.0;         // r^T r
};

// Default-pose prior weights S_kk: the number of vertices with a non-zero
// weight on a link whose chain contains joint k, divided by |V|; zero for the
// joints carrying the root link (a prior pulling the body toward the camera
// origin has no meaning).
inline std::vector<real> prior_weights(const Model& m) {
    std::vector<real> Sk(m.P, 0.0);
    for (int k = 0; k < m.P; ++k) {
        if (m.anc[0][k]) continue;
        int cnt = 0;
        for (int i = 0; i < m.V; ++i) {
            bool hit = false;
            for (int q = 0; q < m.K; ++q) {
                int l = m.skin_link[i * m.K + q];
                if (l >= 0 && m.skin_w[i * m.K + q] > real(0) && m.anc[l][k]) hit = true;
            }
            cnt += hit ? 1 : 0;
        }
        Sk[k] = (real)cnt / (real)m.V;
    }
    return Sk;
}

// Eq. (6)-(8) with the prior: r_i = n_i^T delta_i for i in O = {c_i >= 1,
// |n_i| > 0}; J_i = -n_i^T dv_i/dTheta through dv/dH_Sigma, dH_Sigma/dH_Delta
// (the weight times the identity, with the blend sign) and dH_Delta/dTheta.
inline PoseSystem pose_system(const Model& m, const real* theta, const real* phi, const real* n,
                              const real* delta, const int32_t* cnt, real lambda_s) {
    PoseSystem ps;
    ps.J.assign((size_t)m.V * m.P, 0.0);
    ps.r.assign(m.V, 0.0);
    ps.obs.assign(m.V, 0);
    ps.A.assign((size_t)m.P * m.P, 0.0);
    ps.b.assign(m.P, 0.0);
    auto H = forward_kinematics<real>(m, theta);
    auto H0 = bind_pose<real>(m);
    auto D = link_deltas(m, H, H0);
    // dH_Delta/dtheta blocks per (link, joint)
    std::vector<DQ<real>> dD((size_t)m.L * m.P);
    for (int l = 0; l < m.L; ++l)
        for (int k = 0; k < m.P; ++k)
            if (m.anc[l][k]) dD[(size_t)l * m.P + k] = delta_derivative(m, H, H0, theta, k, l);
    for (int i = 0; i < m.V; ++i) {
        real nl = n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2];
        if (cnt[i] < 1 || nl == real(0)) continue;
        ps.obs[i] = 1;
        ps.r[i] = n[3 * i] * delta[3 * i] + n[3 * i + 1] * delta[3 * i + 1] + n[3 * i + 2] * delta[3 * i + 2];
        real x[3] = {m.rest[3 * i] + phi[3 * i], m.rest[3 * i + 1] + phi[3 * i + 1], m.rest[3 * i + 2] + phi[3 * i + 2]};
        if (m.blend == BLEND_LINEAR) {
            // each influence through its own rigid transform: dv = sum_m w_m dT/dH(H_m, x) dH_m
            real Jm[4][3][8];
            for (int q = 0; q < m.K; ++q) {
                int l = m.skin_link[i * m.K + q];
                if (l >= 0) dq_transform_jacobian(D[l], x, Jm[q]);
            }
            for (int k = 0; k < m.P; ++k) {
                real dv[3] = {0, 0, 0};
                for (int q = 0; q < m.K; ++q) {
                    int l = m.skin_link[i * m.K + q];
                    if (l < 0 || !m.anc[l][k]) continue;
                    const DQ<real>& g = dD[(size_t)l * m.P + k];
                    const real comp[8] = {g.r.w, g.r.x, g.r.y, g.r.z, g.d.w, g.d.x, g.d.y, g.d.z};
                    const real w = m.skin_w[i * m.K + q];
                    for (int d = 0; d < 3; ++d)
                        for (int c = 0; c < 8; ++c) dv[d] += w * Jm[q][d][c] * comp[c];
                }
                ps.J[(size_t)i * m.P + k] = -(n[3 * i] * dv[0] + n[3 * i + 1] * dv[1] + n[3 * i + 2] * dv[2]);
            }
            continue;
        }
        DQ<real> Hs = blend(m, D, i);
        real Jt[3][8];
        dq_transform_jacobian(Hs, x, Jt);
        real sgn[4];
        blend_signs(m, D, i, sgn);
        for (int k = 0; k < m.P; ++k) {
            real dH[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int q = 0; q < m.K; ++q) {
                int l = m.skin_link[i * m.K + q];
                if (l < 0 || !m.anc[l][k]) continue;
                const DQ<real>& g = dD[(size_t)l * m.P + k];
                real w = m.skin_w[i * m.K + q] * sgn[q];
                const real comp[8] = {g.r.w, g.r.x, g.r.y, g.r.z, g.d.w, g.d.x, g.d.y, g.d.z};
                for (int c = 0; c < 8; ++c) dH[c] += w * comp[c];
            }
            real dv[3] = {0, 0, 0};
            for (int d = 0; d < 3; ++d)
                for (int c = 0; c < 8; ++c) dv[d] += Jt[d][c] * dH[c];
            ps.J[(size_t)i * m.P + k] = -(n[3 * i] * dv[0] + n[3 * i + 1] * dv[1] + n[3 * i + 2] * dv[2]);
        }
    }
    // Eq. (7), (8): sums over the observed vertices in index order.
    for (int i = 0; i < m.V; ++i) {
        if (!ps.obs[i]) continue;
        const real* Ji = &ps.J[(size_t)i * m.P];
        for (int k = 0; k < m.P; ++k) {
            ps.b[k] += Ji[k] * ps.r[i];
            for (int q = 0; q < m.P; ++q) ps.A[(size_t)k * m.P + q] += Ji[k] * Ji[q];
        }
        ps.rr += ps.r[i] * ps.r[i];
    }
    // default pose prior: A += (lambda_s S)^2, b += (lambda_s S)^2 Theta
    if (lambda_s != real(0)) {
        auto Sk = prior_weights(m);
        for (int k = 0; k < m.P; ++k) {
            real w = (lambda_s * Sk[k]) * (lambda_s * Sk[k]);
            ps.A[(size_t)k * m.P + k] += w;
            ps.b[k] += w * theta[k];
        }
    }
    return ps;
}

// Damped least squares (Marquardt): (A + lambda_k diag(A)) x = b by Cholesky.
// Parameters with A_kk == 0 exactly (nothing observed moves them) or masked
// inactive are frozen: x_k = 0.  Returns 0, or -4 if the factorisation fails.
inline int lm_solve(int P, const real* A, const real* b, real lambda_k, const uint8_t* active, real* x) {
    std::vector<char> frozen(P, 0);
    for (int k = 0; k < P; ++k) frozen[k] = (A[(size_t)k * P + k] == real(0)) || (active && !active[k]);
    std::vector<real> M((size_t)P * P, 0.0), y(P, 0.0);
    for (int k = 0; k < P; ++k) {
        for (int q = 0; q < P; ++q)
            M[(size_t)k * P + q] = (frozen[k] || frozen[q]) ? real(0) : A[(size_t)k * P + q];
        M[(size_t)k * P + k] = frozen[k] ? real(1) : A[(size_t)k * P + k] * (real(1) + lambda_k);
        y[k] = frozen[k] ? real(0) : b[k];
    }
    // Cholesky M = L L^T (lower triangle stored in place)
    for (int j = 0; j < P; ++j) {
        real s = M[(size_t)j * P + j];
        for (int q = 0; q < j; ++q) s -= M[(size_t)j * P + q] * M[(size_t)j * P + q];
        if (!(s > real(0))) return -4;
        real d = std::sqrt(s);
        M[(size_t)j * P + j] = d;
        for (int i = j + 1; i < P; ++i) {
            real t = M[(size_t)i * P + j];
            for (int q = 0; q < j; ++q) t -= M[(size_t)i * P + q] * M[(size_t)j * P + q];
            M[(size_t)i * P + j] = t / d;
        }
    }
    for (int i = 0; i < P; ++i) {
        real t = y[i];
        for (int q = 0; q < i; ++q) t -= M[(size_t)i * P + q] * x[q];
        x[i] = t / M[(size_t)i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
        real t = x[i];
        for (int q = i + 1; q < P; ++q) t -= M[(size_t)q * P + i] * x[q];
        x[i] = t / M[(size_t)i * P + i];
    }
    for (int k = 0; k < P; ++k) if (frozen[k]) x[k] = 0.0;
    return 0;
}

// ---------------------------------------------------------------------------
// Section 4.3: regularised per-vertex offset update
// ---------------------------------------------------------------------------
// Reading of Eq. (9): the regularisers are separate squared residuals,
//   E_i = r_i^2 + lam_phi |phi_i|^2 + lam_N sum_{n in N(i)} |phi_i - phi_n|^2
//         + lam_T |phi_i - phi_i^prev|^2,
// each vertex takes one damped Gauss-Newton step on its own 3x3 system with
// its neighbours held at their current values (the paper's independence
// approximation), and all vertices update together.  dr_i/dphi_i = -R_i^T n_i
// with R_i the rotation of H_{i,Sigma}; unobserved vertices have no data term.
struct ShapeArgs {
    const real *theta, *phi, *phi_prev, *n, *delta;
    const int32_t* cnt;
    real lambda_phi, lambda_nbr, lambda_t, lambda_w;
};

// Solve the 3x3 system M x = g by Cramer's rule.
inline bool solve3(const real M[9], const real g[3], real x[3]) {
    real c00 = M[4] * M[8] - M[5] * M[7], c01 = M[5] * M[6] - M[3] * M[8], c02 = M[3] * M[7] - M[4] * M[6];
    real det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    if (!(std::fabs(det) > real(0))) return false;
    real inv[9] = {c00, M[2] * M[7] - M[1] * M[8], M[1] * M[5] - M[2] * M[4],
                     c01, M[0] * M[8] - M[2] * M[6], M[2] * M[3] - M[0] * M[5],
                     c02, M[1] * M[6] - M[0] * M[7], M[0] * M[4] - M[1] * M[3]};
    for (int r = 0; r < 3; ++r) x[r] = (inv[3 * r] * g[0] + inv[3 * r + 1] * g[1] + inv[3 * r + 2] * g[2]) / det;
    return true;
}

inline void shape_step(const Model& m, const ShapeArgs& s, real* phi_out) {
    auto H = forward_kinematics<real>(m, s.theta);
    auto H0 = bind_pose<real>(m);
    auto D = link_deltas(m, H, H0);
    for (int i = 0; i < m.V; ++i) {
        const real* ni = &s.n[3 * i];
        real nl = ni[0] * ni[0] + ni[1] * ni[1] + ni[2] * ni[2];
        real u[3] = {0, 0, 0}, r = 0.0;
        if (s.cnt[i] >= 1 && nl > real(0)) {
            real R[9];
            point_jacobian(m, D, i, R);
            for (int c = 0; c < 3; ++c) u[c] = -(R[c] * ni[0] + R[3 + c] * ni[1] + R[6 + c] * ni[2]);
            r = ni[0] * s.delta[3 * i] + ni[1] * s.delta[3 * i + 1] + ni[2] * s.delta[3 * i + 2];
        }
        const real* ph = &s.phi[3 * i];
        real g[3], alpha = s.lambda_phi + s.lambda_t;
        for (int c = 0; c < 3; ++c) g[c] = u[c] * r + s.lambda_phi * ph[c] + s.lambda_t * (ph[c] - s.phi_prev[3 * i + c]);
        for (int q = 0; q < 4; ++q) {
            int j = m.nbr[4 * i + q];
            if (j < 0) continue;
            alpha += s.lambda_nbr;
            for (int c = 0; c < 3; ++c) g[c] += s.lambda_nbr * (ph[c] - s.phi[3 * j + c]);
        }
        real M[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[3 * a + b] = u[a] * u[b] + (a == b ? alpha : real(0));
        for (int a = 0; a < 3; ++a) M[4 * a] *= (real(1) + s.lambda_w);
        real x[3] = {0, 0, 0};
        if (!solve3(M, g, x)) x[0] = x[1] = x[2] = 0.0;
        for (int c = 0; c < 3; ++c) phi_out[3 * i + c] = ph[c] - x[c];
    }
}

// Eq. (9) as printed, kept to show why it is not used: the regularisers sit
// inside one scalar residual per vertex,
//   r^_i = r_i + lam_phi |phi_i|^2 + lam_N sum_{n in N(i)} |phi_i - phi_n|^2,
// its gradient j_i = dr_i/dphi_i + 2 lam_phi phi_i + 2 lam_N sum (phi_i - phi_n)
// is one row, and (j j^T + lam_w diag(j j^T)) x = j r^_i is a rank-one matrix
// plus a diagonal that scales with the squares of j's own entries: its
// solution x_k = r^_i / ((m + lam_w) j_k) (m = non-zero entries of j) grows
// without bound as any entry of j goes to zero.  A singular system (some
// j_k exactly zero) takes no step, as in the reading's solver.
inline void shape_step_literal(const Model& m, const ShapeArgs& s, real* phi_out) {
    auto H = forward_kinematics<real>(m, s.theta);
    auto H0 = bind_pose<real>(m);
    auto D = link_deltas(m, H, H0);
    for (int i = 0; i < m.V; ++i) {
        const real* ni = &s.n[3 * i];
        const real* ph = &s.phi[3 * i];
        real nl = ni[0] * ni[0] + ni[1] * ni[1] + ni[2] * ni[2];
        real j[3] = {0, 0, 0}, r = 0.0;
        if (s.cnt[i] >= 1 && nl > real(0)) {
            real R[9];
            point_jacobian(m, D, i, R);
            for (int c = 0; c < 3; ++c) j[c] = -(R[c] * ni[0] + R[3 + c] * ni[1] + R[6 + c] * ni[2]);
            r = ni[0] * s.delta[3 * i] + ni[1] * s.delta[3 * i + 1] + ni[2] * s.delta[3 * i + 2];
        }
        real rh = r + s.lambda_phi * (ph[0] * ph[0] + ph[1] * ph[1] + ph[2] * ph[2]);
        for (int c = 0; c < 3; ++c) j[c] += real(2) * s.lambda_phi * ph[c];
        for (int q = 0; q < 4; ++q) {
            int k = m.nbr[4 * i + q];
            if (k < 0) continue;
            real d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                real d = ph[c] - s.phi[3 * k + c];
                d2 += d * d;
                j[c] += real(2) * s.lambda_nbr * d;
            }
            rh += s.lambda_nbr * d2;
        }
        real M[9], g[3];
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) M[3 * a + b] = j[a] * j[b];
            M[4 * a] *= (real(1) + s.lambda_w);
            g[a] = j[a] * rh;
        }
        real x[3] = {0, 0, 0};
        if (!solve3(M, g, x)) x[0] = x[1] = x[2] = 0.0;
        for (int c = 0; c < 3; ++c) phi_out[3 * i + c] = ph[c] - x[c];
    }
}

// ---------------------------------------------------------------------------
// Section 4: one frame = n_iters iterations of association, pose step and
// shape step, in that order, with the association kept through the iteration
// ---------------------------------------------------------------------------
struct FrameStats {
    int32_t status, n_valid_px, n_assoc_px, n_obs_verts;
    real energy_first, energy_last, step_norm_last;
};

struct SkinState { std::vector<real> v, n; };

inline SkinState skin_state(const Model& m, const real* theta, const real* phi) {
    SkinState s;
    s.v.resize(3 * m.V);
    s.n.resize(3 * m.V);
    auto H = forward_kinematics<real>(m, theta);
    auto H0 = bind_pose<real>(m);
    auto D = link_deltas(m, H, H0);
    skin(m, D, phi, s.v.data());
    vertex_normals(m, s.v.data(), s.n.data());
    return s;
}

// assoc_in (test hook, may be null): [n_iters * W * H] matches to use in
// place of each iteration's own association, e.g. another implementation's
// choice at pixels whose nearest vertices tie within rounding.
inline int track_frame(const Model& m, const Camera& cam, const Params& prm, real* theta, real* phi,
                       real* phi_prev, const float* depth, const float* xyz, FrameStats* st,
                       real* energies, int32_t* assoc_out, const int32_t* assoc_in = nullptr) {
    const int NP = cam.W * cam.H;
    std::vector<int32_t> a(NP), cnt(m.V);
    std::vector<real> delta(3 * m.V);
    std::vector<float> vf(3 * m.V);
    int n_valid = 0;
    for (int k = 0; k < NP; ++k) { float p[3]; n_valid += point_of_pixel(cam, depth, xyz, k, p) ? 1 : 0; }
    FrameStats s{0, n_valid, 0, 0, 0.0, 0.0, 0.0};
    bool first = true;
    for (int t = 0; t < prm.n_iters; ++t) {
        SkinState ss = skin_state(m, theta, phi);
        for (int q = 0; q < 3 * m.V; ++q) vf[q] = (float)ss.v[q];
        if (assoc_in) std::copy(assoc_in + (size_t)t * NP, assoc_in + (size_t)(t + 1) * NP, a.begin());
        else associate_grid(cam, prm.tau, vf.data(), m.V, depth, xyz, a.data());
        average_offsets(cam, depth, xyz, a.data(), ss.v.data(), m.V, cnt.data(), delta.data());
        int nas = 0, nobs = 0;
        for (int k = 0; k < NP; ++k) nas += a[k] >= 0 ? 1 : 0;
        for (int i = 0; i < m.V; ++i) nobs += cnt[i] > 0 ? 1 : 0;
        s.n_assoc_px = nas;
        s.n_obs_verts = nobs;
        if (assoc_out && t == 0) std::copy(a.begin(), a.end(), assoc_out);
        if (prm.do_pose[t]) {
            PoseSystem ps = pose_system(m, theta, phi, ss.n.data(), delta.data(), cnt.data(), prm.lambda_s);
            if (first) { s.energy_first = ps.rr; first = false; }
            s.energy_last = ps.rr;
            if (energies) energies[t] = ps.rr;
            std::vector<real> x(m.P, 0.0);
            int rc = lm_solve(m.P, ps.A.data(), ps.b.data(), prm.lambda_k,
                              prm.active.empty() ? nullptr : prm.active.data(), x.data());
            if (rc != 0) { s.status = rc; if (st) *st = s; return rc; }
            real nrm = 0.0;
            for (int k = 0; k < m.P; ++k) { theta[k] -= x[k]; nrm += x[k] * x[k]; }
            s.step_norm_last = std::sqrt(nrm);
            SkinState s2 = skin_state(m, theta, phi);
            for (int i = 0; i < m.V; ++i)
                if (cnt[i] > 0)
                    for (int d = 0; d < 3; ++d) delta[3 * i + d] += ss.v[3 * i + d] - s2.v[3 * i + d];
            ss = std::move(s2);
        }
        if (prm.do_shape[t]) {
            std::vector<real> out(3 * m.V);
            ShapeArgs sa{theta, phi, phi_prev, ss.n.data(), delta.data(), cnt.data(),
                         prm.lambda_phi, prm.lambda_nbr, prm.lambda_t, prm.lambda_w};
            shape_step(m, sa, out.data());
            std::copy(out.begin(), out.end(), phi);
        }
    }
    std::copy(phi, phi + 3 * m.V, phi_prev);
    if (st) *st = s;
    return 0;
}

}  // namespace ORC_NS
