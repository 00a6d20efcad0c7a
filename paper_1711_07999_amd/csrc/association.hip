// Projective data association (Section 4.1).
//
// Vertices are projected into pixel buckets (a point-rasterised index kept
// per 4x4-pixel cell, see Buckets) together with each cell's and tile's z
// range (the z-buffer).  Every valid pixel then finds the nearest vertex
// closer than tau: cells are visited in rings around the pixel's cell and
// skipped when a lower bound on the distance of anything inside them (from
// the pixel distance to the cell, or from its z range) cannot beat the best
// distance so far, so the result equals the exhaustive nearest-vertex search.
// The matched offsets are summed per vertex in 64-bit fixed point
// (deterministic).
//
// Float32 decisions follow one operation order, compiled without contraction:
//   point       x = ((u - cx) * d) / fx, y = ((v - cy) * d) / fy, z = d
//   bucket      floor((fx * x) / z + cx + 0.5), floor((fy * y) / z + cy + 0.5)
//   distance    (dx*dx + dy*dy) + dz*dz, accepted if < tau*tau,
//               ties to the lower vertex index.
#include "common.h"
#include "surface.h"

#pragma clang fp contract(off)

namespace trk {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

constexpr uint32_t kInfBits = 0x7F800000u;   // +inf: the z minimum of an empty cell or tile

// ---------------------------------------------------------------------------
// clear both parities' bucket records (counters and layout: every region
// empty, so the first count sends its vertices to the overflow list), the
// per-vertex accumulators and the solve's front image
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_clear(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_CLEAR, blockIdx.x, local)];
    const Buckets& b = S.b;
    const Accum& a = S.a;
    const int V = S.m.V, ntiles = S.c.tiles_x * S.c.tiles_y, ncells = 4 * ntiles;
    const int i = local * blockDim.x + threadIdx.x;
    if (i <= ncells) {
        b.cells[0][i] = make_uint4(kInfBits, 0u, 0u, 0u);
        b.cells[1][i] = make_uint4(kInfBits, 0u, 0u, 0u);
    }
    if (i < ntiles) {
        b.tsum[0][i] = 0u;
        b.tsum[1][i] = 0u;
    }
    if (i < 2) b.ovfn[i] = 0u;
    if (i < 2 * kXcds) b.scnt[i] = 0u;
    if (i < V) {
        a.cnt[i] = 0u;
        a.sx[i] = 0; a.sy[i] = 0; a.sz[i] = 0;
    }
    // the tree solve's front image: zero outside the entries the Gram
    // reduction writes
    if (S.tree.gfmap) {
        const int n = 2 * (ncells + 1) > V ? 2 * (ncells + 1) : V;
        const int stride = (n + 255) / 256 * 256;
        for (int e = i; e < S.tree.elems; e += stride) S.tree.fimg[e] = 0.0;
    }
}

void launch_clear(const Launch& L) {
    launch_kernel(L, true, true, k_clear, dim3(L.grid[KK_CLEAR]), dim3(256), 0, L.B.slots, L.B.pre, L.B.n);
}

// the counters of one parity, its layout kept
__global__ void __launch_bounds__(256) k_clear_counts(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int bsel) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_CLEAR, blockIdx.x, local)];
    const Buckets& b = S.b;
    const int par = S.bpar ^ bsel;
    const int ntiles = S.c.tiles_x * S.c.tiles_y, ncells = 4 * ntiles;
    const int i = local * blockDim.x + threadIdx.x;
    if (i <= ncells) {
        uint4* c = &b.cells[par][i];
        c->x = kInfBits; c->y = 0u; c->z = 0u;
    }
    if (i < ntiles) b.tsum[par][i] = 0u;
    if (i == 0) b.ovfn[par] = 0u;
    if (i < kXcds) b.scnt[par * kXcds + i] = 0u;
}

void launch_clear_counts(const Launch& L, int bsel) {
    launch_kernel(L, true, true, k_clear_counts, dim3(L.grid[KK_CLEAR]), dim3(256), 0, L.B.slots, L.B.pre, L.B.n, bsel);
}

__global__ void __launch_bounds__(256) k_clear_acc(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_VERT, blockIdx.x, local)];
    const int i = local * blockDim.x + threadIdx.x;
    if (i >= S.m.V) return;
    S.a.cnt[i] = 0u;
    S.a.sx[i] = 0; S.a.sy[i] = 0; S.a.sz[i] = 0;
}

void launch_clear_acc(const Launch& L) {
    launch_kernel(L, true, true, k_clear_acc, dim3(L.grid[KK_VERT]), dim3(256), 0, L.B.slots, L.B.pre, L.B.n);
}

// count a given surface into the buckets (the producing kernels count their
// own output instead)
__global__ void __launch_bounds__(256) k_bucket_count(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vsel, int which, int bsel) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_VERT, blockIdx.x, local)];
    if (!selected(S, which)) return;
    const int i = local * blockDim.x + threadIdx.x;
    const bool live = i < S.m.V;
    count_vertex(count_refs(S, bsel), i, S.verts[S.v_cur ^ vsel][live ? i : 0], live, false);
}

void launch_bucket_count(const Launch& L, int vsel, int which, int bsel) {
    launch_kernel(L, true, true, k_bucket_count, dim3(L.grid[KK_VERT]), dim3(256), 0, L.B.slots, L.B.pre, L.B.n, vsel, which, bsel);
}

// ---------------------------------------------------------------------------
// Bucket layout for the next count, from the counts of parity `par`, with
// room for the surface to move: tile t gets d + d/2 + 32 slots, d the largest
// count among the 3x3 tiles around it (so a tile the surface moves into has
// room), placed after the tiles before it; inside it, cell c gets its own
// count n + n/2 + 8 plus a quarter of what the tile has beyond the sum of
// those (the last cell the rest).  Written into the other parity with its
// counters cleared.  A workgroup takes kLayoutTiles tiles (one per thread)
// and sums the shares of all tiles before them itself, from the tile counts
// staged in LDS (read from memory when they do not fit).
// ---------------------------------------------------------------------------
constexpr int kLayoutStage = 8192;   // tile counts staged in LDS (32 KB)

__device__ __forceinline__ uint32_t tile_share(uint32_t d) { return d + (d >> 1) + 32u; }

__device__ __forceinline__ void layout_tiles(const Slot& S, int par, int lblk, uint32_t* stage, uint32_t* sred) {
    const Buckets& b = S.b;
    const int tx = S.c.tiles_x, ty = S.c.tiles_y, ntiles = tx * ty;
    const uint32_t* __restrict__ tin = b.tsum[par];
    const uint4* __restrict__ cin = b.cells[par];
    uint4* __restrict__ cout = b.cells[par ^ 1];
    uint32_t* __restrict__ tout = b.tsum[par ^ 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nthr = blockDim.x, nw = nthr / 64;
    const int t0 = lblk * kLayoutTiles;
    const bool staged = ntiles <= kLayoutStage;
    // this thread's tile: its cells' counts, issued first
    const int t = t0 + threadIdx.x;
    const bool live = t < ntiles;
    const int tl = live ? t : 0;
    uint32_t c4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c4[q] = cin[4 * tl + q].z;
    if (staged) {
        for (int u = threadIdx.x; u < ntiles; u += nthr * 10) {
            uint32_t a[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) a[k] = tin[min(u + nthr * k, ntiles - 1)];
#pragma unroll
            for (int k = 0; k < 10; ++k)
                if (u + nthr * k < ntiles) stage[u + nthr * k] = a[k];
        }
        __syncthreads();
    }
    // largest count of column x over rows y-1..y+1 (0 outside the image);
    // the largest count of the 3x3 tiles around (x, y) is that of columns
    // x-1, x, x+1
    auto column = [&](int x, int y) {
        uint32_t d = 0u;
        if (x >= 0 && x < tx)
            for (int yy = max(y - 1, 0); yy <= min(y + 1, ty - 1); ++yy)
                d = max(d, staged ? stage[yy * tx + x] : tin[yy * tx + x]);
        return d;
    };
    // shares of the tiles before this workgroup's: a contiguous run per
    // thread, walked along its rows with the three columns carried over
    uint32_t part = 0u;
    {
        const int chunk = (t0 + nthr - 1) / nthr;
        int u = threadIdx.x * chunk;
        const int ue = min(u + chunk, t0);
        if (u < ue) {
            int x = u % tx, y = u / tx;
            uint32_t cl = column(x - 1, y), cm = column(x, y), cr = column(x + 1, y);
            for (; u < ue; ++u) {
                part += tile_share(max(cl, max(cm, cr)));
                if (++x == tx) {
                    x = 0;
                    ++y;
                    cl = 0u; cm = column(0, y); cr = column(1, y);
                } else {
                    cl = cm; cm = cr; cr = column(x + 1, y);
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) part += (uint32_t)__shfl_xor((int)part, o);
    // this thread's tile share, scanned over the wave
    const int xl = tl % tx, yl = tl / tx;
    const uint32_t R = live ? tile_share(max(column(xl - 1, yl), max(column(xl, yl), column(xl + 1, yl)))) : 0u;
    uint32_t incl = R;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) { sred[wid] = part; sred[nw + wid] = incl; }
    __syncthreads();
    uint32_t base = 0u;
    for (int w = 0; w < nw; ++w) base += sred[w] + (w < wid ? sred[nw + w] : 0u);
    if (live) {
        // R >= the cells' own shares: d >= the tile's count, and the cells'
        // halves sum to at most the tile's half
        uint32_t own[4], sum = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) { own[q] = c4[q] + (c4[q] >> 1) + 8u; sum += own[q]; }
        const uint32_t extra = (R - sum) >> 2;
        // counts of one count phase sum to at most V, so the regions end by
        // ncap; the clamp only keeps every region inside the buffer
        const uint32_t ncap = (uint32_t)b.ncap;
        uint32_t o = base + incl - R;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cout[4 * t + q] = make_uint4(kInfBits, 0u, 0u, min(o, ncap));
            o += own[q] + extra;
        }
        tout[t] = 0u;
        if (t == ntiles - 1) cout[4 * ntiles] = make_uint4(kInfBits, 0u, 0u, min(base + incl, ncap));
    }
    if (lblk == 0 && threadIdx.x == 0) b.ovfn[par ^ 1] = 0u;
}

// the screen counters the next association uses (the association launch
// clears them: its screen has finished with them, this launch's own are
// the other parity's)
__device__ __forceinline__ void clear_screen_counters(const Buckets& b, int spar) {
    if (threadIdx.x < kXcds) b.scnt[spar * kXcds + threadIdx.x] = 0u;
}

__global__ void __launch_bounds__(kAssocThreads) k_layout(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int bsel) {
    const Batch B{bs, bp, bn};
    __shared__ uint32_t stage[kLayoutStage];
    __shared__ uint32_t sred[2 * (kAssocThreads / 64)];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_LAYOUT, blockIdx.x, local)];
    layout_tiles(S, S.bpar ^ bsel, local, stage, sred);
}

void launch_layout(const Launch& L, int bsel) {
    launch_kernel(L, true, true, k_layout, dim3(L.grid[KK_LAYOUT]), dim3(kAssocThreads), 0, L.B.slots, L.B.pre, L.B.n, bsel);
}

// ---------------------------------------------------------------------------
// association: one wave per 8x8 pixel tile, one pixel per lane
// ---------------------------------------------------------------------------
// Lower bound on the distance from the pixel's point (depth d) to any vertex
// whose bucket is m >= 1 rings away: the vertex's ray makes an angle of at
// least (m - 1/2) pixels with the pixel's ray, so the distance is at least
// d * (m - 1/2) / (f_max * R_max), R_max bounding |(b, 1)| over the image.
// lb_c1 = (1 - 1e-4) / (f_max R_max); the 0.001 and 1e-6 terms absorb the
// float32 rounding of the bucket and of the back-projected point.
__device__ __forceinline__ float ring_lb(const DevCam& c, float d, int m) {
    float t = ((float)m - 0.501f) * c.lb_c1 - 1e-6f;
    return t > 0.0f ? d * t : 0.0f;
}

// z-range test: true if no vertex with z in [zmn, zmx] can have a squared
// distance that beats (or, with no match yet, reaches) the current bound.
__device__ __forceinline__ bool z_pruned(float zmn, float zmx, float pz, float bound, bool found) {
    float g1 = zmn - pz, g2 = pz - zmx;
    float g = fmaxf(g1, g2);
    if (!(g > 0.0f)) return false;
    float g2s = g * g;
    return g2s > bound || (!found && g2s >= bound);
}

// One workgroup per 8x8 tile, two waves per 4x4 quadrant of it (one cell of
// the bucket index), each taking two of its pixel rows.  Lane = pixel (8) x
// slot (8): candidate vertices, loaded coalesced and broadcast through LDS,
// go through the wave eight at a time, each lane comparing its pixel's point
// with the candidate of its slot and keeping the key (d2 bits << 32 | vertex
// id), whose minimum is the nearest vertex with ties to the lower index; the
// slots of a pixel are combined by shuffles.  The search walks square rings
// of cells around the quadrant's own cell.  The same launch also runs the
// layout of the next count (its first workgroups, from the counts read here)
// and the vertex normals of the surface (the workgroups after them).
constexpr int kAssocWaves = kAssocThreads / 64;
constexpr int kAssocPass = 256;   // candidates per pass (LDS per wave: 4 KB)
static_assert(kAssocPass % 32 == 0, "a pass is whole trips of eight slots x four steps");

__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}
__device__ __forceinline__ unsigned long long slot_min(unsigned long long k) {
    k = min_u64(k, __shfl_xor(k, 8));
    k = min_u64(k, __shfl_xor(k, 16));
    return min_u64(k, __shfl_xor(k, 32));
}

// The pixel's point (x, y, z) from the depth image (back-projected) or the
// organised cloud; false if the pixel has no measurement.
__device__ __forceinline__ bool pixel_point(const DevCam& c, const float* __restrict__ depth,
                                            const float* __restrict__ xyz, int u, int v, float& px, float& py,
                                            float& pz) {
#pragma clang fp contract(off)
    px = py = pz = 0.0f;
    if (u >= c.W || v >= c.H) return false;
    const int k = v * c.W + u;
    if (xyz) {
        px = ldg(xyz + 3 * k); py = ldg(xyz + 3 * k + 1); pz = ldg(xyz + 3 * k + 2);
        return isfinite(px) && isfinite(py) && isfinite(pz) && pz > 0.0f;
    }
    const float d = ldg(depth + k);
    if (!(d > 0.0f && isfinite(d))) return false;
    px = (((float)u - c.cx) * d) / c.fx;
    py = (((float)v - c.cy) * d) / c.fy;
    pz = d;
    return true;
}

// Pixel rings that can hold a vertex closer than tau to the wave's points
// (over-estimate is harmless), capped by the image: the widest need of the
// wave's lanes.
__device__ __forceinline__ int window_rings(const DevCam& c, float tau, bool valid, float pz) {
    int rmax = 0;
    if (valid) {
        const int cap = max(c.W, c.H);
        float mf = 0.501f + (tau / pz + 1e-6f) / c.lb_c1;
        rmax = mf >= (float)cap ? cap : (int)mf + 1;
    }
    for (int o = 32; o > 0; o >>= 1) rmax = max(rmax, __shfl_xor(rmax, o));
    return rmax;
}

// Cheap rejection of background: false if no tile of the window (rw pixel
// rings around tile (tx, ty), in whole tiles) has a z range within tau of
// the z range of the wave's points, so nothing can be found.  One tile of
// the window per lane, all loads in flight at once.  A wave with more
// points or a wider window tests a superset.
__device__ __forceinline__ bool window_has_candidates(const DevCam& c, const uint4* __restrict__ cells, float tau,
                                                      int tx, int ty, int rw, bool valid, float pz) {
    const int lane = threadIdx.x & 63;
    bool candidate_tiles = false;
    if (__any(valid)) {
        float pmin = valid ? pz : INFINITY, pmax = valid ? pz : -INFINITY;
        for (int o = 32; o > 0; o >>= 1) {
            pmin = fminf(pmin, __shfl_xor(pmin, o));
            pmax = fmaxf(pmax, __shfl_xor(pmax, o));
        }
        const float tz_tol = tau * 1.0001f + 1e-6f;  // generous: this is only a filter
        const int tr = (rw + 7) / 8;
        const int wx0 = max(tx - tr, 0), wx1 = min(tx + tr, c.tiles_x - 1);
        const int wy0 = max(ty - tr, 0), wy1 = min(ty + tr, c.tiles_y - 1);
        const int nwx = wx1 - wx0 + 1, nwin = nwx * (wy1 - wy0 + 1);
        for (int base = 0; base < nwin && !candidate_tiles; base += 64) {
            const int qw = base + lane;
            bool cand = false;
            if (qw < nwin) {
                const int wy = qw / nwx;
                // the tile's z range from its four cells' (an empty cell
                // holds (+inf, 0): an empty tile is never a candidate)
                const uint2* cz = reinterpret_cast<const uint2*>(cells + 4 * ((wy0 + wy) * c.tiles_x + wx0 + (qw - wy * nwx)));
                const uint2 r0 = ldg(cz), r1 = ldg(cz + 2), r2 = ldg(cz + 4), r3 = ldg(cz + 6);
                const float zlo = __uint_as_float(min(min(r0.x, r1.x), min(r2.x, r3.x)));
                const float zhi = __uint_as_float(max(max(r0.y, r1.y), max(r2.y, r3.y)));
                cand = zlo <= zhi && zlo < pmax + tz_tol && zhi > pmin - tz_tol;
            }
            candidate_tiles = __any(cand);
        }
    }
    return candidate_tiles;
}

// The search of one part of a tile -- two pixel rows of one of its 4x4
// quadrants (part = 2 quadrant + row pair) -- by one wave with an LDS buffer
// of kAssocPass candidates: the pixels' matches, the per-vertex sums, and
// the part's counts of (valid, matched, newly observed) pixels.
__device__ __forceinline__ int3 search_part(const Slot& S, int par, int vsel, int tile, int part, float4* cand) {
    const DevCam& c = S.c;
    const Buckets& b = S.b;
    const uint4* __restrict__ cells = b.cells[par];
    // the overflow list: compared whole, once, by a wave that needs one of
    // the cells whose region was full
    const uint32_t novf = min(b.ovfn[par], (uint32_t)S.m.V);
    // held in scalar registers: read through the slot inside the copy loops,
    // they would be reloaded after every copy into LDS (which the compiler
    // takes as a store that may alias them), each reload waiting for every
    // copy still in flight
    const float4* __restrict__ cellv = wave_uniform(b.cellv);
    const uint32_t ovf_at = wave_uniform((uint32_t)b.ncap);
    const Accum& a = S.a;
    const float tau = S.tau;
    const float4* __restrict__ verts = S.verts[S.v_cur ^ vsel];
    int32_t* __restrict__ assoc = S.assoc;
    const int lane = wave_lane();
    const int tx = tile % c.tiles_x, ty = tile / c.tiles_x;
    const int q = lane & 7, slot = lane >> 3, quad = part >> 1, rows = 2 * (part & 1);
    const int ccx = 2 * tx + (quad & 1), ccy = 2 * ty + (quad >> 1);   // the quadrant's cell
    const int u = ccx * 4 + (q & 3), v = ccy * 4 + rows + (q >> 2);
    const bool inimg = u < c.W && v < c.H;
    float px, py, pz;
    const bool valid = pixel_point(c, S.depth, S.xyz, u, v, px, py, pz);
    const float tau2 = tau * tau;
    const uint32_t tau2_bits = __float_as_uint(tau2);
    // key of the best candidate so far (this slot's, and the pixel's as of
    // the last finished ring); an unmatched valid pixel holds (tau^2, 0),
    // which no candidate at distance >= tau can undercut, an invalid one 0,
    // which nothing undercuts
    unsigned long long key = valid ? ((unsigned long long)tau2_bits << 32) : 0ull;
    unsigned long long best = key;
    // pixel rings that can hold a vertex closer than tau (over-estimate is
    // harmless), capped by the image; the wave's widest need sets the cells
    const int rw = window_rings(c, tau, valid, pz);
    // rings 0..Rc of cells cover every pixel within 4 Rc of the quadrant
    const int Rc = (rw + 3) / 4 + 1;
    bool done = !valid;
    const int cells_x = 2 * c.tiles_x, cells_y = 2 * c.tiles_y;
    // cheap rejection of background (see window_has_candidates)
    const bool candidate_tiles = window_has_candidates(c, cells, tau, tx, ty, rw, valid, pz);
    if (candidate_tiles) {
        // The cells of the (2 Rc + 1)^2 square around the quadrant's cell, in
        // ring order (ring R >= 1, the perimeter of the (2R+1)^2 square,
        // starts at entry (2R-1)^2), come 64 at a time, one record per lane.
        // A block is searched in batches -- in the first block, rings 0 and 1
        // (entries 0..8) first, then the rest -- and a batch takes every cell
        // some pixel still needs under the bound left by the batches before,
        // loading all of its candidates before comparing any.
        bool ovf_done = false;
        auto run_batch = [&](unsigned long long cellmask, unsigned long long ovfcells, const uint4& rec, int rcx,
                             int rcy) {
            // lane = cell: is it needed by one of the wave's 8 pixels (the
            // pixel-distance and z-range bounds cannot exclude a better vertex)?
            // A finished pixel counts with bound 0, which excludes everything.
            const uint32_t bbits = done ? 0u : (uint32_t)(best >> 32);
            const float c_zmn = __uint_as_float(rec.z), c_zmx = __uint_as_float(rec.w);
            const int X0 = rcx * 4, Y0 = rcy * 4;
            bool need = false;
#pragma unroll
            for (int pq = 0; pq < 8; ++pq) {
                const int up = ccx * 4 + (pq & 3), vp = ccy * 4 + rows + (pq >> 2);
                const float pzp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pz), pq));
                const uint32_t bp = (uint32_t)__builtin_amdgcn_readlane((int)bbits, pq);
                const float bound = __uint_as_float(bp);
                const int mx = max(max(X0 - up, up - (X0 + 3)), 0), my = max(max(Y0 - vp, vp - (Y0 + 3)), 0);
                const float lb = ring_lb(c, pzp, max(mx, my));
                need = need || (!(lb * lb >= bound) && !z_pruned(c_zmn, c_zmx, pzp, bound, bp < tau2_bits));
            }
            const unsigned long long needed = __ballot(need) & cellmask;
            const bool take_ovf = !ovf_done && (needed & ovfcells) != 0ull;
            uint32_t total = take_ovf ? novf : 0u;
            for (unsigned long long m = needed; m; m &= m - 1ull)
                total += (uint32_t)__builtin_amdgcn_readlane((int)rec.y, __builtin_ctzll(m));
            // the needed cells' candidates in cell order, up to kAssocPass per
            // pass, copied from the sorted vertices straight into LDS (one DMA
            // load per cell, all in flight together); every pixel compares
            // every candidate (extra candidates are real vertices: the minimum
            // stays exact)
            for (uint32_t pass = 0; pass < total; pass += kAssocPass) {
                const uint32_t pend = pass + (uint32_t)kAssocPass;
                uint32_t pre = 0u;
                // candidates [off, off + cnt) of `cellv` as the segment after `pre`
                auto segment = [&](uint32_t off, uint32_t cnt) {
                    const uint32_t a0 = max(pre, pass), a1 = min(pre + cnt, pend);
                    for (uint32_t s0 = a0; s0 < a1; s0 += 64u) {
                        if ((uint32_t)lane < a1 - s0)
                            __builtin_amdgcn_global_load_lds(
                                (const void*)(cellv + (off + (s0 - pre) + (uint32_t)lane)),
                                (__attribute__((address_space(3))) void*)&cand[s0 - pass], 16, 0, 0);
                    }
                    pre += cnt;
                };
                for (unsigned long long m = needed; m; m &= m - 1ull) {
                    const int k = __builtin_ctzll(m);
                    segment((uint32_t)__builtin_amdgcn_readlane((int)rec.x, k),
                            (uint32_t)__builtin_amdgcn_readlane((int)rec.y, k));
                    if (pre >= pend) break;   // the rest belongs to later passes
                }
                if (take_ovf && pre < pend) segment(ovf_at, novf);
                const int n = (int)min((uint32_t)kAssocPass, total - pass);
                // the pass's last trip filled up with entries at x = +inf: for a
                // finite pixel their d2 is +inf or NaN, whose bits no key of a
                // valid pixel (at most tau^2, 0) or of an invalid one (0) exceeds
                const int ntrip = (n + 31) & ~31;
                if (lane < ntrip - n) cand[n + lane].x = __builtin_inff();
                __builtin_amdgcn_s_waitcnt(0);   // the copies have landed in LDS
                __builtin_amdgcn_wave_barrier();
                // eight slots x four steps per trip, the LDS reads issued together
                for (int i0 = 0; i0 < ntrip; i0 += 32) {
                    float4 sv[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) sv[j] = cand[i0 + 8 * j + slot];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float dx = sv[j].x - px, dy = sv[j].y - py, dz = sv[j].z - pz;
                        const float d2 = (dx * dx + dy * dy) + dz * dz;
                        const unsigned long long kk =
                            ((unsigned long long)__float_as_uint(d2) << 32) | (uint32_t)__float_as_int(sv[j].w);
                        key = kk < key ? kk : key;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
            if (take_ovf) ovf_done = true;
            best = slot_min(key);
        };
        const int last = (2 * Rc + 1) * (2 * Rc + 1);
        for (int cur = 0; cur < last; cur += 64) {
            const int l2 = cur + lane;
            int sq = (int)sqrtf((float)l2);
            while ((sq + 1) * (sq + 1) <= l2) ++sq;
            while (sq * sq > l2) --sq;
            const int rr = (sq + 1) >> 1;
            // (first slot, vertices in the region, zmin bits, zmax bits)
            uint4 myrec = make_uint4(0u, 0u, 0u, 0u);
            uint32_t mycnt = 0u;
            int mycx = 0, mycy = 0;
            if (l2 < last) {
                const int kq = rr == 0 ? 0 : l2 - (2 * rr - 1) * (2 * rr - 1);
                const int side = 2 * rr + 1;
                if (rr == 0) { mycx = ccx; mycy = ccy; }
                else if (kq < side) { mycx = ccx - rr + kq; mycy = ccy - rr; }
                else if (kq < 2 * side) { mycx = ccx - rr + (kq - side); mycy = ccy + rr; }
                else if (kq < 3 * side - 2) { mycx = ccx - rr; mycy = ccy - rr + 1 + (kq - 2 * side); }
                else { mycx = ccx + rr; mycy = ccy - rr + 1 + (kq - (3 * side - 2)); }
                if (mycx >= 0 && mycy >= 0 && mycx < cells_x && mycy < cells_y) {
                    const int ci = (((mycy >> 1) * c.tiles_x + (mycx >> 1)) << 2) | ((mycy & 1) << 1) | (mycx & 1);
                    const uint4 r = ldg(cells + ci);
                    const uint32_t end = ldg(&cells[ci + 1].w);
                    const uint32_t cap = end > r.w ? end - r.w : 0u;
                    mycnt = r.z;
                    myrec = make_uint4(r.w, min(r.z, cap), r.x, r.y);
                }
            }
            const unsigned long long todo = __ballot(mycnt != 0u);
            const unsigned long long ovfc = __ballot(mycnt > myrec.y);
            if (cur == 0) {
                run_batch(todo & 0x1FFull, ovfc, myrec, mycx, mycy);
                run_batch(todo & ~0x1FFull, ovfc, myrec, mycx, mycy);
            } else {
                run_batch(todo, ovfc, myrec, mycx, mycy);
            }
            // the complete rings so far; every cell outside their square is
            // at least m_next pixels away
            const int end = min(cur + 64, last);
            int Rd = 0;
            while ((2 * Rd + 3) * (2 * Rd + 3) <= end) ++Rd;
            if (!done) {
                const int X0b = (ccx - Rd) * 4, X1b = (ccx + Rd) * 4 + 3;
                const int Y0b = (ccy - Rd) * 4, Y1b = (ccy + Rd) * 4 + 3;
                const int m_next = min(min(u - X0b, X1b - u), min(v - Y0b, Y1b - v)) + 1;
                const float lb = ring_lb(c, pz, m_next);
                done = lb * lb >= __uint_as_float((uint32_t)(best >> 32));
            }
            if (__all(done)) break;
        }
    }
    key = slot_min(key);
    // slot 0 lanes hold the pixels
    int bestv = -1;
    bool first = false;
    const bool mine = slot == 0;
    if (mine && valid && (uint32_t)(key >> 32) < tau2_bits) {
        bestv = (int)(uint32_t)key;
        const float4 sv = ldg_xyz(verts + bestv);
        const float dx = sv.x - px, dy = sv.y - py, dz = sv.z - pz;
        uint32_t old = atomic_add_g(a.cnt + bestv, 1u);
        atomic_add_g((unsigned long long*)&a.sx[bestv], (unsigned long long)(long long)rintf(-dx * 4294967296.0f));
        atomic_add_g((unsigned long long*)&a.sy[bestv], (unsigned long long)(long long)rintf(-dy * 4294967296.0f));
        atomic_add_g((unsigned long long*)&a.sz[bestv], (unsigned long long)(long long)rintf(-dz * 4294967296.0f));
        first = old == 0u;
    }
    if (mine && inimg) stg(assoc + v * c.W + u, bestv);
    const unsigned long long vb = __ballot(mine && valid), ab = __ballot(bestv >= 0), fb = __ballot(first);
    return make_int3(__popcll(vb), __popcll(ab), __popcll(fb));
}

// Tiles where nothing can match are finished by the screen (one wave per
// tile); the others are queued for the search workgroups of the XCD the
// screen ran on, or, when that queue is full, searched by the screen wave
// itself, part by part.
// (held to eight waves per SIMD: its own work is a few loads and a test; the
// registers of the rare search of a tile beyond its queue spill instead)
__global__ void __launch_bounds__(64, 8) k_assoc_screen(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vsel, int bsel, int sflip) {
    const Batch B{bs, bp, bn};
    __shared__ float4 scand1[kAssocPass];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_SCREEN, blockIdx.x, local)];
    const DevCam& c = S.c;
    const Buckets& b = S.b;
    const int par = S.bpar ^ bsel, spar = par ^ sflip;
    const int tile = b.torder[local];
    if (tile < 0) return;   // an XCD with fewer tiles than the others
    const int lane = threadIdx.x;
    const int tx = tile % c.tiles_x, ty = tile / c.tiles_x;
    const int u = 8 * tx + (lane & 7), v = 8 * ty + (lane >> 3);
    float px, py, pz;
    const bool valid = pixel_point(c, S.depth, S.xyz, u, v, px, py, pz);
    // the tile's 64 points together: their z range and rings bound those of
    // every wave that would search a part of the tile
    const int rw = window_rings(c, S.tau, valid, pz);
    if (!window_has_candidates(c, b.cells[par], S.tau, tx, ty, rw, valid, pz)) {
        if (u < c.W && v < c.H) S.assoc[v * c.W + u] = -1;
        const int nv = __popcll(__ballot(valid));
        if (lane == 0) b.bstat[tile] = make_int4(nv, 0, 0, 0);
        return;
    }
    const int x = local % kXcds;   // this workgroup's XCD
    uint32_t at = 0u;
    if (lane == 0) at = atomicAdd(&b.scnt[spar * kXcds + x], 1u);
    at = (uint32_t)__builtin_amdgcn_readfirstlane((int)at);
    if (at < (uint32_t)b.capx) {
        if (lane == 0) b.tlist[x * b.capx + at] = tile;
        return;
    }
    int4 t = make_int4(0, 0, 0, 0);
    for (int part = 0; part < kAssocWaves; ++part) {
        const int3 r = search_part(S, par, vsel, tile, part, scand1);
        t.x += r.x; t.y += r.y; t.z += r.z;
    }
    if (lane == 0) b.bstat[tile] = t;
}

__global__ void __launch_bounds__(kAssocThreads, 8) k_associate(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vsel, int bsel, int sflip, int queued) {
    const Batch B{bs, bp, bn};
    __shared__ float4 scand[kAssocWaves][kAssocPass];
    __shared__ int4 scount[kAssocWaves];
    int local;
    const Slot& S = B.slots[slot_of(B, queued ? KK_ASSOCQ : KK_ASSOC, blockIdx.x, local)];
    const DevCam& c = S.c;
    const Buckets& b = S.b;
    const int par = S.bpar ^ bsel;
    {
        const int nlay = layout_blocks(c.tiles_x * c.tiles_y), nnorm = assoc_normal_blocks(S.m.V);
        if (local < nlay) {
            static_assert(sizeof(scand) >= kLayoutStage * sizeof(uint32_t), "layout stage fits the candidate LDS");
            if (local == 0) clear_screen_counters(b, par ^ sflip ^ 1);
            layout_tiles(S, par, local, reinterpret_cast<uint32_t*>(&scand[0][0]), reinterpret_cast<uint32_t*>(scount));
            return;
        }
        if (local < nlay + nnorm) {
            const int i = (local - nlay) * kAssocThreads + threadIdx.x;
            const bool live = i < S.m.V;
            float nx, ny, nz;
            vertex_normal_lean(S.m, S.verts[S.v_cur ^ vsel], i, live, nx, ny, nz);   // the whole wave
            if (live) { S.normals.x[i] = nx; S.normals.y[i] = ny; S.normals.z[i] = nz; }
            return;
        }
        // workgroups rounding the extras up to a multiple of kXcds: none
        const int nextra = assoc_extra_blocks(c.tiles_x * c.tiles_y, S.m.V);
        if (local < nextra) return;
        local -= nextra;
    }
    int tile;
    if (queued) {
        // workgroup k (on XCD k % 8) takes entry k / 8 of that XCD's queue
        const int x = local % kXcds, at = local / kXcds;
        const uint32_t nq = min(b.scnt[(par ^ sflip) * kXcds + x], (uint32_t)b.capx);
        if ((uint32_t)at >= nq) return;
        tile = b.tlist[x * b.capx + at];
    } else {
        tile = b.torder[local];
        if (tile < 0) return;   // an XCD with fewer tiles than the others
    }
    const int wid = threadIdx.x >> 6;
    const int3 r = search_part(S, par, vsel, tile, wid, scand[wid]);
    // per-workgroup counts go to this workgroup's own slot (no shared counter:
    // device-wide atomics on one address serialise across the chip)
    if ((threadIdx.x & 63) == 0) scount[wid] = make_int4(r.x, r.y, r.z, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        int4 t = scount[0];
        for (int w = 1; w < kAssocWaves; ++w) { t.x += scount[w].x; t.y += scount[w].y; t.z += scount[w].z; }
        b.bstat[tile] = t;
    }
}

void launch_associate(const Launch& L, int vsel, int bsel, int sflip) {
    // A single stream is bound by its longest searches, which start at once
    // with every tile's workgroup in flight; a batch is bound by the total
    // work, most of it the background tiles' workgroups, which the screen
    // finishes with a wave each.
    if (L.B.n == 1) {
        launch_kernel(L, true, true, k_associate, dim3(L.grid[KK_ASSOC]), dim3(kAssocThreads), 0, L.B.slots, L.B.pre, L.B.n, vsel, bsel,
                      sflip, 0);
        return;
    }
    launch_kernel(L, true, false, k_assoc_screen, dim3(L.grid[KK_SCREEN]), dim3(64), 0, L.B.slots, L.B.pre, L.B.n, vsel, bsel, sflip);
    launch_kernel(L, false, true, k_associate, dim3(L.grid[KK_ASSOCQ]), dim3(kAssocThreads), 0, L.B.slots, L.B.pre, L.B.n, vsel, bsel,
                  sflip, 1);
}

}  // namespace trk
