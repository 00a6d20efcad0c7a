// Quaternion and dual-quaternion arithmetic on the device (Section 3.1).
// A dual quaternion H = r + eps d is held as 8 numbers: r.w r.x r.y r.z,
// d.w d.x d.y d.z.
#pragma once
#include <hip/hip_runtime.h>

namespace trk {

template <class T>
__device__ __forceinline__ void qmul(const T* a, const T* b, T* o) {
    T w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    T x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    T y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    T z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

// o = a * b for dual quaternions: (a.r b.r, a.r b.d + a.d b.r)
template <class T>
__device__ __forceinline__ void dqmul(const T* a, const T* b, T* o) {
    T r[4], d1[4], d2[4];
    qmul(a, b, r);
    qmul(a, b + 4, d1);
    qmul(a + 4, b, d2);
    o[0] = r[0]; o[1] = r[1]; o[2] = r[2]; o[3] = r[3];
    o[4] = d1[0] + d2[0]; o[5] = d1[1] + d2[1]; o[6] = d1[2] + d2[2]; o[7] = d1[3] + d2[3];
}

// Conjugate of both parts; the inverse of a unit dual quaternion.
template <class T>
__device__ __forceinline__ void dqconj(const T* a, T* o) {
    o[0] = a[0]; o[1] = -a[1]; o[2] = -a[2]; o[3] = -a[3];
    o[4] = a[4]; o[5] = -a[5]; o[6] = -a[6]; o[7] = -a[7];
}

// Point transform by a possibly non-unit (blended) dual quaternion:
//   T(H, x) = (r x r* + 2 vec(d r*)) / |r|^2,
// with r x r* = (w^2 - q.q) x + 2 (q.x) q + 2 w (q cross x) for r = (w, q)
// and vec(d r*) = w d_v - d_w q + q cross d_v.
__device__ __forceinline__ void dq_apply(const float* H, float x, float y, float z, float& ox,
                                         float& oy, float& oz) {
    float w = H[0], qx = H[1], qy = H[2], qz = H[3];
    float dw = H[4], dx = H[5], dy = H[6], dz = H[7];
    float qq = qx * qx + qy * qy + qz * qz;
    float nn = w * w + qq;
    float s = w * w - qq;
    float qdx = qx * x + qy * y + qz * z;
    float cx = qy * z - qz * y, cy = qz * x - qx * z, cz = qx * y - qy * x;
    float ax = s * x + 2.0f * qdx * qx + 2.0f * w * cx;
    float ay = s * y + 2.0f * qdx * qy + 2.0f * w * cy;
    float az = s * z + 2.0f * qdx * qz + 2.0f * w * cz;
    float ex = qy * dz - qz * dy, ey = qz * dx - qx * dz, ez = qx * dy - qy * dx;
    float bx = w * dx - dw * qx + ex;
    float by = w * dy - dw * qy + ey;
    float bz = w * dz - dw * qz + ez;
    float inv = 1.0f / nn;
    ox = (ax + 2.0f * bx) * inv;
    oy = (ay + 2.0f * by) * inv;
    oz = (az + 2.0f * bz) * inv;
}

// Blend of up to four link offsets with the weights of one vertex, each
// signed to the hemisphere of the largest-weight influence (ties: lower
// link index).  dq holds 8 floats per link.
__device__ __forceinline__ void dq_blend(const float* dq, float4 w, uint32_t links, float* H,
                                         float* sgn_out = nullptr) {
    const float ws[4] = {w.x, w.y, w.z, w.w};
    int piv = -1;
    float wb = -1.0f;
    int lb = 0x7fffffff;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int l = (links >> (8 * k)) & 0xFF;
        if (l == 0xFF) continue;
        if (ws[k] > wb || (ws[k] == wb && l < lb)) { wb = ws[k]; lb = l; piv = l; }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) H[c] = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int l = (links >> (8 * k)) & 0xFF;
        float sg = 1.0f;
        if (l != 0xFF) {
            const float* a = dq + 8 * l;
            const float* p = dq + 8 * piv;
            float d = a[0] * p[0] + a[1] * p[1] + a[2] * p[2] + a[3] * p[3];
            sg = d < 0.0f ? -1.0f : 1.0f;
            float ww = ws[k] * sg;
#pragma unroll
            for (int c = 0; c < 8; ++c) H[c] += ww * a[c];
        }
        if (sgn_out) sgn_out[k] = sg;
    }
}

// The linear variant of the blend (matrix linear blend skinning): the point
// moved rigidly by each influence's unit link offset, averaged with the
// weights.  No hemisphere signs: each link's motion is applied on its own.
__device__ __forceinline__ void lbs_apply(const float* dq, float4 w, uint32_t links, float x, float y, float z,
                                          float& ox, float& oy, float& oz) {
    const float ws[4] = {w.x, w.y, w.z, w.w};
    ox = 0.0f; oy = 0.0f; oz = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int l = (links >> (8 * k)) & 0xFF;
        if (l == 0xFF) continue;
        float tx, ty, tz;
        dq_apply(dq + 8 * l, x, y, z, tx, ty, tz);
        ox += ws[k] * tx;
        oy += ws[k] * ty;
        oz += ws[k] * tz;
    }
}

// Rotation matrix (row-major) of the quaternion r / |r|.
template <class T>
__device__ __forceinline__ void quat_matrix(const float* q, T R[9]) {
    const T w = q[0], x = q[1], y = q[2], z = q[3];
    const T s = T(2) / (w * w + x * x + y * y + z * z);
    R[0] = T(1) - s * (y * y + z * z); R[1] = s * (x * y - w * z); R[2] = s * (x * z + w * y);
    R[3] = s * (x * y + w * z); R[4] = T(1) - s * (x * x + z * z); R[5] = s * (y * z - w * x);
    R[6] = s * (x * z - w * y); R[7] = s * (y * z + w * x); R[8] = T(1) - s * (x * x + y * y);
}

}  // namespace trk
