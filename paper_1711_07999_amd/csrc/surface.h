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
    }
    // tile sums: neighbouring vertices share tiles, so the lanes of a wave
    // are grouped by tile and one lane per tile adds the group's count
    const int tile = pix >= 0 ? (pix >> 6) : -1;
    unsigned long long todo = __ballot(tile >= 0);
    while (todo) {
        const int t0 = __builtin_amdgcn_readlane(tile, __builtin_ctzll(todo));
        const unsigned long long grp = __ballot(tile == t0);
        if (tile == t0 && (threadIdx.x & 63) == __builtin_ctzll(grp)) atomicAdd(&b.tsum[t0], (uint32_t)__popcll(grp));
        todo &= ~grp;
    }
}

// A vertex's own position and its inline fan (the loads that wait on
// nothing), so that a caller can issue them with its other first reads.
struct FanIn {
    float4 p;
    uint32_t e0, e1;
    int2 bc[kFanInline];
};

__device__ __forceinline__ void vertex_fan_load(const DevModel& m, const float4* __restrict__ v, int i, bool live,
                                                FanIn& f) {
    f.p = v[live ? i : 0];
    f.e0 = live ? m.fan_off[i] : 0u;
    f.e1 = live ? m.fan_off[i + 1] : 0u;
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) f.bc[k] = live ? m.fan8[(size_t)k * m.V + i] : make_int2(0, 0);
}

// Sum over the incident faces (b, c) of (v_b - v_i) x (v_c - v_i),
// normalised; zero if the sum vanishes.  One operation order (no
// contraction) wherever it is inlined, so every kernel gets the same bits:
// the first kFanInline faces in fan order from the inline table (its padding
// entries (i, i) add an exact zero; all loads issued at once), then, for a
// vertex of more faces, the rest summed by the whole wave (lane l takes
// faces l, l + 64, ... of the rest; a fixed tree adds the lanes' sums).
// Every lane of the wave must call it together.  This form takes the loads
// made by vertex_fan_load (with a `live` at least as wide as this one);
// lanes with live == false gather nothing of their own (their result is not
// meaningful) but take part in the shared work.
__device__ __forceinline__ void vertex_normal_fan(const DevModel& m, const float4* __restrict__ v, int i, bool live,
                                                  const FanIn& f, float& nx, float& ny, float& nz) {
#pragma clang fp contract(off)
    const int ii = live ? i : 0;
    const float4 p = f.p;
    const uint32_t e0 = live ? f.e0 : 0u, e1 = live ? f.e1 : 0u;
    int2 bc[kFanInline];
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) bc[k] = live ? f.bc[k] : make_int2(0, 0);
    float4 vb[kFanInline], vc[kFanInline];
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) { vb[k] = v[bc[k].x]; vc[k] = v[bc[k].y]; }
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) {
        const float ax = vb[k].x - p.x, ay = vb[k].y - p.y, az = vb[k].z - p.z;
        const float bx = vc[k].x - p.x, by = vc[k].y - p.y, bz = vc[k].z - p.z;
        sx += ay * bz - az * by;
        sy += az * bx - ax * bz;
        sz += ax * by - ay * bx;
    }
    const int lane = threadIdx.x & 63;
    for (unsigned long long h = __ballot(live && e1 - e0 > (uint32_t)kFanInline); h; h &= h - 1ull) {
        const int k = __builtin_ctzll(h);
        const int hv = __builtin_amdgcn_readlane(ii, k);
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)e0, k) + kFanInline;
        const uint32_t z = (uint32_t)__builtin_amdgcn_readlane((int)e1, k);
        const float4 ph = v[hv];
        float tx = 0.0f, ty = 0.0f, tz = 0.0f;
        for (uint32_t e = a + (uint32_t)lane; e < z; e += 64u) {
            const int2 f = m.fan[e];
            const float4 b = v[f.x], c = v[f.y];
            const float ax = b.x - ph.x, ay = b.y - ph.y, az = b.z - ph.z;
            const float bx = c.x - ph.x, by = c.y - ph.y, bz = c.z - ph.z;
            tx += ay * bz - az * by;
            ty += az * bx - ax * bz;
            tz += ax * by - ay * bx;
        }
        for (int o = 32; o > 0; o >>= 1) {
            tx += __shfl_down(tx, o);
            ty += __shfl_down(ty, o);
            tz += __shfl_down(tz, o);
        }
        const float ex = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tx), 0));
        const float ey = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ty), 0));
        const float ez = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tz), 0));
        if (lane == k) { sx += ex; sy += ey; sz += ez; }
    }
    const float l = sqrtf(sx * sx + sy * sy + sz * sz);
    const float inv = l > 0.0f ? 1.0f / l : 0.0f;
    nx = sx * inv; ny = sy * inv; nz = sz * inv;
}

__device__ __forceinline__ void vertex_normal(const DevModel& m, const float4* __restrict__ v, int i, bool live,
                                              float& nx, float& ny, float& nz) {
    FanIn f;
    vertex_fan_load(m, v, i, live, f);
    vertex_normal_fan(m, v, i, live, f, nx, ny, nz);
}

}  // namespace trk
