// Per-vertex pieces shared by the kernels that produce or consume a skinned
// surface: the vertex's bucket in the point-rasterised index (Section 4.1)
// and its area-weighted normal.
#pragma once
#include "common.h"

namespace trk {

// pixel (u, v) -> its bucket: 8x8 tiles in row-major order, Morton order
// inside a tile (so every 4x4 quadrant of a tile is 16 consecutive buckets)
__device__ __forceinline__ int tile_pixel(int tiles_x, int u, int v) {
    const int m = (u & 1) | ((v & 1) << 1) | ((u & 2) << 1) | ((v & 2) << 2) | ((u & 4) << 2) | ((v & 4) << 3);
    return (((v >> 3) * tiles_x + (u >> 3)) << 6) + m;
}

// What a count reads of its slot, read before the kernel's first global
// store and held in scalar registers: read after a store, each field would
// be reloaded and waited for on its own.
struct CountRefs {
    uint4* cells;       // the counters bsel selects
    uint32_t* tsum;
    uint32_t* ovfn;
    float4* cellv;
    int* status;
    float fx, fy, cx, cy;
    int W, H, tiles_x;
    uint32_t ncap, V;
};

__device__ __forceinline__ CountRefs count_refs(const Slot& S, int bsel) {
    const int par = S.bpar ^ bsel;
    CountRefs r;
    r.cells = wave_uniform(S.b.cells[par]);
    r.tsum = wave_uniform(S.b.tsum[par]);
    r.ovfn = wave_uniform(S.b.ovfn + par);
    r.cellv = wave_uniform(S.b.cellv);
    r.status = wave_uniform(&S.st->status);
    r.fx = wave_uniform(S.c.fx);
    r.fy = wave_uniform(S.c.fy);
    r.cx = wave_uniform(S.c.cx);
    r.cy = wave_uniform(S.c.cy);
    r.W = wave_uniform(S.c.W);
    r.H = wave_uniform(S.c.H);
    r.tiles_x = wave_uniform(S.c.tiles_x);
    r.ncap = wave_uniform((uint32_t)S.b.ncap);
    r.V = wave_uniform((uint32_t)S.m.V);
    return r;
}

// Bucket of vertex i at p (float32 decisions in one fixed order, no
// contraction):  floor((fx * x) / z + cx + 0.5), floor((fy * y) / z + cy + 0.5)
// for z > kZNear inside the image, else none.  Counts the vertex into its
// cell and tile of the counters bsel selects; unless count_only, also into
// the cell's z range, and stores (x, y, z, i) in the cell's region, or in
// the overflow list when the region is full.  Every lane of the wave calls
// it together: the lanes that share a cell (or tile) are grouped and take
// one atomic per counter (a cell's vertices come from many waves, so
// per-lane atomics on it would queue behind each other).
__device__ __forceinline__ void count_vertex(const CountRefs& R, int i, float4 p, bool live, bool count_only) {
#pragma clang fp contract(off)
    uint4* __restrict__ cells = R.cells;
    const int lane = threadIdx.x & 63;
    int pix = -1;
    if (live && p.z > kZNear) {
        const float fu = floorf((R.fx * p.x) / p.z + R.cx + 0.5f);
        const float fv = floorf((R.fy * p.y) / p.z + R.cy + 0.5f);
        if (fu >= 0.0f && fu < (float)R.W && fv >= 0.0f && fv < (float)R.H) pix = tile_pixel(R.tiles_x, (int)fu, (int)fv);
    }
    const int cell = pix >= 0 ? (pix >> 4) : -1;
    if (count_only) {
        uint32_t gsize = 0u;
        for (unsigned long long todo = __ballot(cell >= 0); todo;) {
            const int lead = __builtin_ctzll(todo);
            const int c0 = __builtin_amdgcn_readlane(cell, lead);
            const unsigned long long grp = __ballot(cell == c0);
            if (lane == lead) gsize = (uint32_t)__popcll(grp);
            todo &= ~grp;
        }
        if (gsize != 0u) atomic_add_g(&cells[cell].z, gsize);
    } else {
        // the region's bounds do not wait for the slot (unconditional loads:
        // a lane with no cell reads cell 0's and drops them)
        const int cc = cell >= 0 ? cell : 0;
        const uint32_t off0 = ldg(&cells[cc].w), end0 = ldg(&cells[cc + 1].w);
        const uint32_t off = cell >= 0 ? off0 : 0u, end = cell >= 0 ? end0 : 0u;
        const uint32_t zb = __float_as_uint(p.z);  // z > 0: integer order is float order
        // per cell: the group's first lane gets the group's size and z range
        // (the z range one lane at a time on the scalar unit: a group is a
        // few lanes); then every group's first lane adds them at once (the
        // slot base returns into that lane: one round trip for the wave,
        // not one per group).  A lane's slot is its leader's base plus its
        // rank in the group.
        uint32_t gsize = 0u, gmn = 0xFFFFFFFFu, gmx = 0u;
        int leader = lane, rank = 0;
        const unsigned long long below = (1ull << lane) - 1ull;
        for (unsigned long long todo = __ballot(cell >= 0); todo;) {
            const int lead = __builtin_ctzll(todo);
            const int c0 = __builtin_amdgcn_readlane(cell, lead);
            const unsigned long long grp = __ballot(cell == c0);
            uint32_t mn = 0xFFFFFFFFu, mx = 0u;
            for (unsigned long long m = grp; m; m &= m - 1ull) {
                const uint32_t z = (uint32_t)__builtin_amdgcn_readlane((int)zb, __builtin_ctzll(m));
                mn = min(mn, z);
                mx = max(mx, z);
            }
            if (lane == lead) { gsize = (uint32_t)__popcll(grp); gmn = mn; gmx = mx; }
            if (cell == c0) { leader = lead; rank = __popcll(grp & below); }
            todo &= ~grp;
        }
        uint32_t base = 0u;
        if (gsize != 0u) {
            base = atomic_add_g(&cells[cell].z, gsize);
            atomic_min_g(&cells[cell].x, gmn);
            atomic_max_g(&cells[cell].y, gmx);
        }
        const uint32_t slot = (uint32_t)__shfl((int)base, leader) + (uint32_t)rank;
        if (cell >= 0) {
            const float4 rec = make_float4(p.x, p.y, p.z, __int_as_float(i));
            if (slot < (end > off ? end - off : 0u)) {
                stg(R.cellv + off + slot, rec);
            } else {
                // at most V entries between two clears of the counters; more
                // would mean a count into counters nobody cleared: the frame
                // is failed rather than a vertex dropped
                const uint32_t o = atomic_add_g(R.ovfn, 1u);
                if (o < R.V) stg(R.cellv + R.ncap + o, rec);
                else *R.status = kStatusBucketOverflow;
            }
        }
    }
    // tile counts, grouped the same way
    uint32_t* __restrict__ tsum = R.tsum;
    const int tile = pix >= 0 ? (pix >> 6) : -1;
    uint32_t tsize = 0u;
    for (unsigned long long todo = __ballot(tile >= 0); todo;) {
        const int lead = __builtin_ctzll(todo);
        const int t0 = __builtin_amdgcn_readlane(tile, lead);
        const unsigned long long grp = __ballot(tile == t0);
        if (lane == lead) tsize = (uint32_t)__popcll(grp);
        todo &= ~grp;
    }
    if (tsize != 0u) atomic_add_g(tsum + tile, tsize);
}

// The faces past the inline table (vertices of more than kFanInline faces,
// summed by the whole wave: lane l takes faces l, l + 64, ... of the rest; a
// fixed tree adds the lanes' sums), added to (sx, sy, sz), then normalised.
__device__ __forceinline__ void fan_rest_and_normalise(const DevModel& m, const float4* __restrict__ v, int ii,
                                                       bool live, uint32_t e0, uint32_t e1, float sx, float sy,
                                                       float sz, float& nx, float& ny, float& nz) {
#pragma clang fp contract(off)
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

// A vertex's own position and its inline fan (the loads that wait on
// nothing), so that a caller can issue them with its other first reads.
struct FanIn {
    float4 p;
    uint32_t e0, e1;
    int2 bc[kFanInline];
};

__device__ __forceinline__ void vertex_fan_load(const DevModel& m, const float4* __restrict__ v, int i, bool live,
                                                FanIn& f) {
    // every load unconditional (lanes past the end read vertex 0's entries),
    // so that none waits under a branch for the one before it, and global,
    // so that a wait for LDS does not wait for them
    const int ii = live ? i : 0;
    f.p = ldg_xyz(v + ii);
    f.e0 = ldg(m.fan_off + ii);
    f.e1 = ldg(m.fan_off + ii + 1);
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) f.bc[k] = ldg(m.fan8 + (size_t)k * m.V + ii);
}

// The loads of vertex_fan_load held where this stands (waited for here, not
// moved under the branches that use them) and dropped for lanes not live.
__device__ __forceinline__ void vertex_fan_settle(FanIn& f, bool live) {
    pin_load(f.e0);
    pin_load(f.e1);
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) pin_load(f.bc[k]);
    f.e0 = live ? f.e0 : 0u;
    f.e1 = live ? f.e1 : 0u;
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) f.bc[k] = live ? f.bc[k] : make_int2(0, 0);
}

// Sum over the incident faces (b, c) of (v_b - v_i) x (v_c - v_i),
// normalised; zero if the sum vanishes.  One operation order (no
// contraction) wherever it is inlined, so every kernel gets the same bits:
// the first kFanInline faces in fan order from the inline table (its padding
// entries (i, i) add an exact zero; all loads issued at once), then, for a
// vertex of more faces, the rest summed by the whole wave (lane l takes
// faces l, l + 64, ... of the rest; a fixed tree adds the lanes' sums).
// Every lane of the wave must call it together.  This form takes the loads
// made by vertex_fan_load and vertex_fan_settle (with a `live` at least as
// wide as this one);
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
    for (int k = 0; k < kFanInline; ++k) { vb[k] = ldg_xyz(v + bc[k].x); vc[k] = ldg_xyz(v + bc[k].y); }
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) {
        const float ax = vb[k].x - p.x, ay = vb[k].y - p.y, az = vb[k].z - p.z;
        const float bx = vc[k].x - p.x, by = vc[k].y - p.y, bz = vc[k].z - p.z;
        sx += ay * bz - az * by;
        sy += az * bx - ax * bz;
        sz += ax * by - ay * bx;
    }
    fan_rest_and_normalise(m, v, ii, live, e0, e1, sx, sy, sz, nx, ny, nz);
}

// The same normal with fewer registers live: the inline fan's vertices are
// gathered two faces a round (for a kernel that must stay within 64
// registers).
__device__ __forceinline__ void vertex_normal_lean(const DevModel& m, const float4* __restrict__ v, int i, bool live,
                                                   float& nx, float& ny, float& nz) {
#pragma clang fp contract(off)
    const int ii = live ? i : 0;
    const float4 p = v[ii];
    // unconditional loads (vertex 0's entries past the end): none waits
    // under a branch for the one before it
    uint32_t f0 = m.fan_off[ii], f1 = m.fan_off[ii + 1];
    int2 bcs[kFanInline];
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) bcs[k] = m.fan8[(size_t)k * m.V + ii];
    pin_load(f0);
    pin_load(f1);
#pragma unroll
    for (int k = 0; k < kFanInline; ++k) {
        pin_load(bcs[k]);
        bcs[k] = live ? bcs[k] : make_int2(0, 0);
    }
    const uint32_t e0 = live ? f0 : 0u, e1 = live ? f1 : 0u;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int k0 = 0; k0 < kFanInline; k0 += 2) {
        // no gather of a later round is moved above this one (registers)
        __builtin_amdgcn_sched_barrier(0);
        float4 vb[2], vc[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int2 bc = bcs[k0 + k];
            vb[k] = v[bc.x];
            vc[k] = v[bc.y];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float ax = vb[k].x - p.x, ay = vb[k].y - p.y, az = vb[k].z - p.z;
            const float bx = vc[k].x - p.x, by = vc[k].y - p.y, bz = vc[k].z - p.z;
            sx += ay * bz - az * by;
            sy += az * bx - ax * bz;
            sz += ax * by - ay * bx;
        }
    }
    fan_rest_and_normalise(m, v, ii, live, e0, e1, sx, sy, sz, nx, ny, nz);
}

__device__ __forceinline__ void vertex_normal(const DevModel& m, const float4* __restrict__ v, int i, bool live,
                                              float& nx, float& ny, float& nz) {
    FanIn f;
    vertex_fan_load(m, v, i, live, f);
    vertex_fan_settle(f, live);
    vertex_normal_fan(m, v, i, live, f, nx, ny, nz);
}

}  // namespace trk
