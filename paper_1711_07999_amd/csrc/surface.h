// Per-vertex pieces shared by the kernels that produce or consume a skinned
// surface: the vertex's bucket in the point-rasterised index (Section 4.1)
// and its area-weighted normal.
#pragma once
#include "common.h"

namespace trk {

// pixel (u, v) -> its bucket: 8x8 tiles in row-major order, Morton order
// inside a tile (so every 4x4 quadrant of a tile is 16 consecutive buckets)
__device__ __forceinline__ int tile_pixel(const DevCam& c, int u, int v) {
    const int m = (u & 1) | ((v & 1) << 1) | ((u & 2) << 1) | ((v & 2) << 2) | ((u & 4) << 2) | ((v & 4) << 3);
    return (((v >> 3) * c.tiles_x + (u >> 3)) << 6) + m;
}

// Bucket of vertex i at p (float32 decisions in one fixed order, no
// contraction):  floor((fx * x) / z + cx + 0.5), floor((fy * y) / z + cy + 0.5)
// for z > kZNear inside the image, else none.  Counts the vertex into its
// pixel (rank kept for the scatter), the pixel's z range and the tile's sum.
__device__ __forceinline__ void count_vertex(const Slot& S, int i, float4 p) {
#pragma clang fp contract(off)
    const DevCam& c = S.c;
    const Buckets& b = S.b;
    int pix = -1;
    if (p.z > kZNear) {
        const float fu = floorf((c.fx * p.x) / p.z + c.cx + 0.5f);
        const float fv = floorf((c.fy * p.y) / p.z + c.cy + 0.5f);
        if (fu >= 0.0f && fu < (float)c.W && fv >= 0.0f && fv < (float)c.H) pix = tile_pixel(c, (int)fu, (int)fv);
    }
    b.vpix[i] = pix;
    if (pix >= 0) {
        b.vslot[i] = atomicAdd(&b.pcnt[pix], 1u);
        const uint32_t zb = __float_as_uint(p.z);  // z > 0: integer order is float order
        atomicMin(&b.pzmin[pix], zb);
        atomicMax(&b.pzmax[pix], zb);
        atomicAdd(&b.tsum[pix >> 6], 1u);
    }
}

// Sum over the incident faces (b, c) of (v_b - v_i) x (v_c - v_i), in fan
// order, normalised; zero if the sum vanishes.  One operation order (no
// contraction) wherever it is inlined, so every kernel gets the same bits.
__device__ __forceinline__ void vertex_normal(const DevModel& m, const float4* __restrict__ v, int i, float& nx,
                                              float& ny, float& nz) {
#pragma clang fp contract(off)
    const float4 p = v[i];
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    const uint32_t e1 = m.fan_off[i + 1];
    for (uint32_t e = m.fan_off[i]; e < e1; ++e) {
        const int2 bc = m.fan[e];
        const float4 vb = v[bc.x], vc = v[bc.y];
        const float ax = vb.x - p.x, ay = vb.y - p.y, az = vb.z - p.z;
        const float bx = vc.x - p.x, by = vc.y - p.y, bz = vc.z - p.z;
        sx += ay * bz - az * by;
        sy += az * bx - ax * bz;
        sz += ax * by - ay * bx;
    }
    const float l = sqrtf(sx * sx + sy * sy + sz * sz);
    const float inv = l > 0.0f ? 1.0f / l : 0.0f;
    nx = sx * inv; ny = sy * inv; nz = sz * inv;
}

}  // namespace trk
