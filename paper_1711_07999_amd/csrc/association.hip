// Projective data association (Section 4.1).
//
// Vertices are projected into per-pixel buckets (a point-rasterised index
// buffer kept as a counting sort) together with each bucket's z range (the
// z-buffer).  Every valid pixel then searches rings of buckets around itself
// for the nearest vertex closer than tau, stopping as soon as a lower bound on
// the distance of anything in the next ring exceeds the best distance, so the
// result equals the exhaustive nearest-vertex search.  The matched offsets are
// summed per vertex in 64-bit fixed point (deterministic).
//
// Float32 decisions follow one operation order, compiled without contraction:
//   point       x = ((u - cx) * d) / fx, y = ((v - cy) * d) / fy, z = d
//   bucket      floor((fx * x) / z + cx + 0.5), floor((fy * y) / z + cy + 0.5)
//   distance    (dx*dx + dy*dy) + dz*dz, accepted if < tau*tau,
//               ties to the lower vertex index.
#include "common.h"

#pragma clang fp contract(off)

namespace trk {

__device__ __forceinline__ int tile_pixel(const DevCam& c, int u, int v) {
    return (((v >> 3) * c.tiles_x + (u >> 3)) << 6) + ((v & 7) << 3) + (u & 7);
}

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// ---------------------------------------------------------------------------
// clear the bucket counters, z ranges, per-vertex accumulators and counters
// ---------------------------------------------------------------------------
__global__ void k_clear(int npad, Buckets b, int V, Accum a, DevStats* st) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) {
        b.pcnt[i] = 0u;
        b.pzmin[i] = 0x7F800000u;  // +inf
        b.pzmax[i] = 0u;
    }
    if (i < V) {
        a.cnt[i] = 0u;
        a.sx[i] = 0; a.sy[i] = 0; a.sz[i] = 0;
    }
    if (i == 0) { st->n_valid_px = 0; st->n_assoc_px = 0; st->n_obs_verts = 0; }
}

void launch_clear(hipStream_t s, int npad, const Buckets& b, int V, const Accum& a, DevStats* st) {
    int n = npad > V ? npad : V;
    hipLaunchKernelGGL(k_clear, dim3((n + 255) / 256), dim3(256), 0, s, npad, b, V, a, st);
}

// ---------------------------------------------------------------------------
// bucket construction: count -> per-tile sums and z ranges -> tile prefix ->
// per-pixel offsets -> scatter
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bucket_count(DevCam c, int V, CVec3Buf v, Buckets b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    float x = v.x[i], y = v.y[i], z = v.z[i];
    int pix = -1;
    if (z > kZNear) {
        float fu = floorf((c.fx * x) / z + c.cx + 0.5f);
        float fv = floorf((c.fy * y) / z + c.cy + 0.5f);
        if (fu >= 0.0f && fu < (float)c.W && fv >= 0.0f && fv < (float)c.H)
            pix = tile_pixel(c, (int)fu, (int)fv);
    }
    b.vpix[i] = pix;
    if (pix >= 0) {
        b.vslot[i] = atomicAdd(&b.pcnt[pix], 1u);
        uint32_t zb = __float_as_uint(z);  // z > 0: integer order is float order
        atomicMin(&b.pzmin[pix], zb);
        atomicMax(&b.pzmax[pix], zb);
    }
}

// one wave per tile
__global__ void __launch_bounds__(256) k_tile_reduce(int ntiles, Buckets b) {
    int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    int p = (tile << 6) + wave_lane();
    uint32_t cnt = b.pcnt[p];
    float zmn = __uint_as_float(b.pzmin[p]);
    float zmx = cnt ? __uint_as_float(b.pzmax[p]) : -INFINITY;
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o);
        zmn = fminf(zmn, __shfl_xor(zmn, o));
        zmx = fmaxf(zmx, __shfl_xor(zmx, o));
    }
    if (wave_lane() == 0) {
        b.tsum[tile] = cnt;
        b.tz[tile] = make_float2(zmn, zmx);
    }
}

// exclusive prefix over tiles, one workgroup of 1024 threads
__global__ void __launch_bounds__(1024) k_tile_scan(int ntiles, Buckets b) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = wave_lane(), wid = threadIdx.x >> 6;
    for (int base = 0; base < ntiles; base += 1024) {
        int i = base + threadIdx.x;
        uint32_t x = i < ntiles ? b.tsum[i] : 0u;
        uint32_t incl = x;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        uint32_t wpre = 0, total = 0;
        for (int w = 0; w < 16; ++w) {
            uint32_t s = wsum[w];
            if (w < wid) wpre += s;
            total += s;
        }
        if (i < ntiles) b.toff[i] = carry + wpre + incl - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
}

// per-pixel (offset, count, zmin, zmax); one wave per tile
__global__ void __launch_bounds__(256) k_pixel_offsets(int ntiles, Buckets b) {
    int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int lane = wave_lane();
    int p = (tile << 6) + lane;
    uint32_t cnt = b.pcnt[p];
    uint32_t incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    b.rec[p] = make_uint4(b.toff[tile] + incl - cnt, cnt, b.pzmin[p], b.pzmax[p]);
}

__global__ void __launch_bounds__(256) k_bucket_scatter(int V, CVec3Buf v, Buckets b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    int pix = b.vpix[i];
    if (pix < 0) return;
    uint32_t dst = b.rec[pix].x + b.vslot[i];
    b.sorted[dst] = make_float4(v.x[i], v.y[i], v.z[i], __int_as_float(i));
}

void launch_bucket(hipStream_t s, const DevCam& c, int V, CVec3Buf v, const Buckets& b) {
    int ntiles = c.tiles_x * c.tiles_y;
    hipLaunchKernelGGL(k_bucket_count, dim3((V + 255) / 256), dim3(256), 0, s, c, V, v, b);
    hipLaunchKernelGGL(k_tile_reduce, dim3((ntiles + 3) / 4), dim3(256), 0, s, ntiles, b);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, ntiles, b);
    hipLaunchKernelGGL(k_pixel_offsets, dim3((ntiles + 3) / 4), dim3(256), 0, s, ntiles, b);
    hipLaunchKernelGGL(k_bucket_scatter, dim3((V + 255) / 256), dim3(256), 0, s, V, v, b);
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

__global__ void __launch_bounds__(256) k_associate(DevCam c, float tau, const float* __restrict__ depth,
                                                   const float* __restrict__ xyz, Buckets b, Accum a,
                                                   int32_t* __restrict__ assoc, DevStats* st) {
    const int ntiles = c.tiles_x * c.tiles_y;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int lane = wave_lane();
    const int tx = tile % c.tiles_x, ty = tile / c.tiles_x;
    const int u = tx * 8 + (lane & 7), v = ty * 8 + (lane >> 3);
    const bool inimg = u < c.W && v < c.H;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    bool valid = false;
    if (inimg) {
        int k = v * c.W + u;
        if (xyz) {
            px = xyz[3 * k]; py = xyz[3 * k + 1]; pz = xyz[3 * k + 2];
            valid = isfinite(px) && isfinite(py) && isfinite(pz) && pz > 0.0f;
        } else {
            float d = depth[k];
            valid = d > 0.0f && isfinite(d);
            if (valid) {
                px = (((float)u - c.cx) * d) / c.fx;
                py = (((float)v - c.cy) * d) / c.fy;
                pz = d;
            }
        }
    }
    const float tau2 = tau * tau;
    int best = -1;
    float bd2 = tau2, bdx = 0.0f, bdy = 0.0f, bdz = 0.0f;
    if (valid) {
        // rings that can hold a vertex closer than tau
        int rmax = 0;
        while (rmax < kRhoCap && ring_lb(c, pz, rmax + 1) < tau) ++rmax;
        // whole-window test on the tile z ranges (cheap rejection of background)
        int u0 = max(u - rmax, 0), u1 = min(u + rmax, c.W - 1);
        int v0 = max(v - rmax, 0), v1 = min(v + rmax, c.H - 1);
        bool any = false;
        for (int ty2 = v0 >> 3; ty2 <= (v1 >> 3) && !any; ++ty2)
            for (int tx2 = u0 >> 3; tx2 <= (u1 >> 3); ++tx2) {
                float2 tz = b.tz[ty2 * c.tiles_x + tx2];
                if (!z_pruned(tz.x, tz.y, pz, tau2, false)) { any = true; break; }
            }
        if (any) {
            for (int rho = 0; rho <= rmax; ++rho) {
                const int nring = rho == 0 ? 1 : 8 * rho;
                for (int q = 0; q < nring; ++q) {
                    int uu, vv;
                    if (rho == 0) { uu = u; vv = v; }
                    else if (q < 2 * rho + 1) { uu = u - rho + q; vv = v - rho; }
                    else if (q < 4 * rho + 2) { uu = u - rho + (q - 2 * rho - 1); vv = v + rho; }
                    else if (q < 6 * rho + 1) { uu = u - rho; vv = v - rho + 1 + (q - 4 * rho - 2); }
                    else { uu = u + rho; vv = v - rho + 1 + (q - 6 * rho - 1); }
                    if (uu < 0 || vv < 0 || uu >= c.W || vv >= c.H) continue;
                    uint4 r = b.rec[tile_pixel(c, uu, vv)];
                    if (r.y == 0u) continue;
                    if (z_pruned(__uint_as_float(r.z), __uint_as_float(r.w), pz, bd2, best >= 0)) continue;
                    for (uint32_t e = r.x; e < r.x + r.y; ++e) {
                        float4 s = b.sorted[e];
                        float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
                        float d2 = (dx * dx + dy * dy) + dz * dz;
                        int id = __float_as_int(s.w);
                        if (d2 < bd2 || (d2 == bd2 && best >= 0 && id < best)) {
                            best = id; bd2 = d2; bdx = dx; bdy = dy; bdz = dz;
                        }
                    }
                }
                float lb = ring_lb(c, pz, rho + 1);
                if (lb * lb >= bd2) break;
            }
        }
        if (best >= 0) {
            uint32_t old = atomicAdd(&a.cnt[best], 1u);
            atomicAdd((unsigned long long*)&a.sx[best], (unsigned long long)(long long)rintf(-bdx * 4294967296.0f));
            atomicAdd((unsigned long long*)&a.sy[best], (unsigned long long)(long long)rintf(-bdy * 4294967296.0f));
            atomicAdd((unsigned long long*)&a.sz[best], (unsigned long long)(long long)rintf(-bdz * 4294967296.0f));
            if (old == 0u) atomicAdd(&st->n_obs_verts, 1);
        }
    }
    if (inimg) assoc[v * c.W + u] = best;
    unsigned long long vb = __ballot(valid), ab = __ballot(best >= 0);
    if (lane == 0) {
        if (vb) atomicAdd(&st->n_valid_px, __popcll(vb));
        if (ab) atomicAdd(&st->n_assoc_px, __popcll(ab));
    }
}

void launch_associate(hipStream_t s, const DevCam& c, float tau, const float* depth, const float* xyz,
                      const Buckets& b, const Accum& a, int32_t* assoc, DevStats* st) {
    int ntiles = c.tiles_x * c.tiles_y;
    hipLaunchKernelGGL(k_associate, dim3((ntiles + 3) / 4), dim3(256), 0, s, c, tau, depth, xyz, b, a,
                       assoc, st);
}

}  // namespace trk
