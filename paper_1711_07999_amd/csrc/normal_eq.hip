// Residuals, pose Jacobian rows and the normal equations (Eq. 6-8).
//
// For each observed vertex i (at least one associated pixel and a non-zero
// normal) the residual is r_i = n_i . delta_i with delta_i the mean offset of
// its points (Eq. 6).  Its Jacobian row follows the chain rule of Section 4.2;
// with dH_{l,Delta}/dtheta_k = Xi_k H_{l,Delta} (see the FK kernel) and
// dT/dH collapsed against the normal into one dual quaternion c = (c_r, c_d),
//   c_d = (2/N) n r,   c_r = -(2/N) (n r x + n d + (n . v) r),   N = |r|^2
// for the blend H = (r, d), template point x = v0 + phi and skinned point v,
// every entry is a dot product of 6-vectors:
//   J_ik = - sum over influences m whose link chain holds joint k of
//          w_m [ vec(c_r H_m,r^* + c_d H_m,d^*) . Xi_k,r + vec(c_d H_m,r^*) . Xi_k,d ].
// Rows are built in LDS as [J | r] (never written to HBM) and the Gram matrix
// G = [J r]^T [J r] (which holds J^T J, J^T r and r^T r) is accumulated with
// MFMA with float32 accumulation, from one of three operand forms:
//   mode 0: float32 operands (v_mfma_f32_16x16x4_f32);
//   mode 1: each entry split as hi + lo in bfloat16, G ~ hi.hi + hi.lo + lo.hi
//           (3 bfloat16 products, about 2^-17 relative error per product);
//   mode 2: hi + mid + lo, G ~ hi.hi + hi.mid + mid.hi + hi.lo + lo.hi + mid.mid
//           (6 products, about 2^-24: float32 accuracy at bfloat16 rate).
// Each workgroup writes one partial G; partials are summed in workgroup
// order (deterministic) by a second kernel.
#include "common.h"
#include "dq.h"

namespace trk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kJTStride = kNeRows + 8;  // floats per LDS column of the row tile
constexpr int kGStride = 25;            // floats per row of per-influence 6-vectors
constexpr int kNeWaves = 8;             // waves per chunk's workgroup
constexpr int kNeThreads = 64 * kNeWaves;
// upper 16x16 Gram blocks each wave owns at most
constexpr int kNeBlocks = ((kPPMax / 16) * (kPPMax / 16 + 1) / 2 + kNeWaves - 1) / kNeWaves;

__device__ __forceinline__ void block_of(int idx, int nb, int& I, int& J) {
    int q = idx;
    for (I = 0; I < nb; ++I) {
        int len = nb - I;
        if (q < len) { J = I + q; return; }
        q -= len;
    }
    I = J = 0;
}

// what a vertex's row needs, read in one round of loads
struct VertexIn {
    float4 w, v;
    uint32_t links, cnt;
    float nx, ny, nz, x0, x1, x2;   // normal; template point + offset
    long long sx, sy, sz;           // fixed-point sums of its points' offsets
};

__device__ __forceinline__ void vertex_load(const DevModel& m, int i, const float4* v, const Vec3Buf& n,
                                            const Vec3Buf& phi, const Accum& a, VertexIn& in) {
    // global reads: as flat reads they would also count as LDS and scalar
    // accesses, and the first wait for one of those would wait for them
    in.w = ldg(m.w + i);
    in.links = ldg(m.links + i);
    in.v = ldg(v + i);
    in.nx = ldg(n.x + i); in.ny = ldg(n.y + i); in.nz = ldg(n.z + i);
    in.cnt = ldg(a.cnt + i);
    in.sx = (long long)ldg(a.sx + i); in.sy = (long long)ldg(a.sy + i); in.sz = (long long)ldg(a.sz + i);
    const float rx = ldg(m.rx + i), ry = ldg(m.ry + i), rz = ldg(m.rz + i);
    const float px = ldg(phi.x + i), py = ldg(phi.y + i), pz = ldg(phi.z + i);
    // every read issued before the first use of one
    __builtin_amdgcn_sched_barrier(0);
    in.x0 = rx + px;
    in.x1 = ry + py;
    in.x2 = rz + pz;
}

// per-vertex 6-vectors of the Jacobian (one per influence) and the residual
__device__ __forceinline__ void vertex_terms(const float* sdq, const VertexIn& in, float* G, float& r_out,
                                             bool linear) {
    float H[8], sg[4];
    const float4 w = in.w;
    const uint32_t lk = in.links;
    const float inv = 1.0f / ((float)in.cnt * 4294967296.0f);
    const float dx = (float)in.sx * inv, dy = (float)in.sy * inv, dz = (float)in.sz * inv;
    if (linear) {
        // the linear blend: influence m moves the template point rigidly to
        // y_m = T(H_m, x), and dy_m/dtheta_k = Xi_k acting on y_m, so its
        // 6-vector is 2 w_m (y_m x n, n) (the one-influence case of the
        // collapsed form above)
        const float nx = in.nx, ny = in.ny, nz = in.nz;
        const float ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int l = (lk >> (8 * k)) & 0xFF;
            float* g = G + 6 * k;
            if (l == 0xFF) {
                g[0] = g[1] = g[2] = g[3] = g[4] = g[5] = 0.0f;
                continue;
            }
            float yx, yy, yz;
            dq_apply(sdq + 8 * l, in.x0, in.x1, in.x2, yx, yy, yz);
            const float s2 = 2.0f * ws[k];
            g[0] = s2 * (yy * nz - yz * ny);
            g[1] = s2 * (yz * nx - yx * nz);
            g[2] = s2 * (yx * ny - yy * nx);
            g[3] = s2 * nx;
            g[4] = s2 * ny;
            g[5] = s2 * nz;
        }
        r_out = nx * dx + ny * dy + nz * dz;
        return;
    }
    dq_blend(sdq, w, lk, H, sg);
    const float nx = in.nx, ny = in.ny, nz = in.nz;
    const float vx = in.v.x, vy = in.v.y, vz = in.v.z;
    const float x[4] = {0.0f, in.x0, in.x1, in.x2};
    const float nq[4] = {0.0f, nx, ny, nz};
    const float N = H[0] * H[0] + H[1] * H[1] + H[2] * H[2] + H[3] * H[3];
    const float s2 = 2.0f / N;
    float nr[4], nrx[4], nd[4];
    qmul(nq, H, nr);
    qmul(nr, x, nrx);
    qmul(nq, H + 4, nd);
    const float ndotv = nx * vx + ny * vy + nz * vz;
    float cr[4], cd[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cd[c] = s2 * nr[c];
        cr[c] = -s2 * (nrx[c] + nd[c] + ndotv * H[c]);
    }
    const float ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int l = (lk >> (8 * k)) & 0xFF;
        float* g = G + 6 * k;
        if (l == 0xFF) {
            g[0] = g[1] = g[2] = g[3] = g[4] = g[5] = 0.0f;
            continue;
        }
        const float* D = sdq + 8 * l;
        const float s = sg[k];
        const float rc[4] = {s * D[0], -s * D[1], -s * D[2], -s * D[3]};
        const float dc[4] = {s * D[4], -s * D[5], -s * D[6], -s * D[7]};
        float t1[4], t2[4], t3[4];
        qmul(cr, rc, t1);
        qmul(cd, dc, t2);
        qmul(cd, rc, t3);
        const float ww = ws[k];
        g[0] = ww * (t1[1] + t2[1]);
        g[1] = ww * (t1[2] + t2[2]);
        g[2] = ww * (t1[3] + t2[3]);
        g[3] = ww * t3[1];
        g[4] = ww * t3[2];
        g[5] = ww * t3[3];
    }
    r_out = nx * dx + ny * dy + nz * dz;
}

// Dynamic LDS of the normal equations for the batch's largest padded size
// ppmax and link count lmax: the [col][row] tile (float32, or two / three
// bfloat16 planes), the per-row 6-vectors, links, residuals and the staged
// link offsets, generators and link chains.  Sized to the batch so that a
// 75-joint body stays under 64 KB (larger workgroup LDS costs launch time).
template <int MODE>
__host__ __device__ inline size_t ne_tile_bytes(int ppmax) {
    return (size_t)ppmax * kJTStride * (MODE == 0 ? 4 : MODE == 1 ? 4 : 6);
}
template <int MODE>
__host__ __device__ inline size_t ne_lds_bytes(int ppmax, int lmax) {
    return ne_tile_bytes<MODE>(ppmax) + 4 * (size_t)kNeRows * kGStride + 4 * (size_t)kNeRows * 2 + 48 +
           4 * (size_t)(8 * lmax + 6 * ppmax + 4 * lmax);
}

// BIG: an instance allowed more than 64 KB of LDS (hi/mid/lo planes, or
// P > 79); smaller sizes use the other instance, which launches faster
template <int MODE, bool BIG>
__global__ void __launch_bounds__(kNeThreads) k_normal_eq(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vsel, int pn, int ppmax, int lmax) {
    const Batch B{bs, bp, bn};
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    unsigned char* q0 = smem;
    // [col][row] tile: float32 (mode 0) or two / three bfloat16 planes
    float* sJT = reinterpret_cast<float*>(q0);
    __bf16* plane0 = reinterpret_cast<__bf16*>(q0);
    __bf16* plane1 = plane0 + ppmax * kJTStride;
    __bf16* plane2 = plane1 + ppmax * kJTStride;
    q0 += ne_tile_bytes<MODE>(ppmax);
    float* sG = reinterpret_cast<float*>(q0);
    q0 += 4 * kNeRows * kGStride;
    uint32_t* slink = reinterpret_cast<uint32_t*>(q0);
    q0 += 4 * kNeRows;
    float* sr = reinterpret_cast<float*>(q0);
    q0 += 4 * kNeRows;
    int* scount = reinterpret_cast<int*>(q0);
    uint32_t* smask = reinterpret_cast<uint32_t*>(q0 + 16);   // [2][4] columns the waves' rows touch
    q0 += 48;
    float* sdq = reinterpret_cast<float*>(q0);
    q0 += 4 * 8 * lmax;
    float* sxi = reinterpret_cast<float*>(q0);
    q0 += 4 * 6 * ppmax;
    uint32_t* sanc = reinterpret_cast<uint32_t*>(q0);

    int wg;
    const Slot& S = B.slots[slot_of(B, KK_NE, blockIdx.x, wg)];
    const DevModel& m = S.m;
    const int PP = S.PP;
    const float* __restrict__ dq = S.dq;
    const float* __restrict__ xi = S.xi;
    const uint32_t* __restrict__ anc = S.anc;
    const float4* __restrict__ v = S.verts[S.v_cur ^ vsel];
    const Vec3Buf n = S.normals;
    const Vec3Buf phi = S.phi[phi_index(S, pn)];
    const Accum& a = S.a;
    const int nchunks = (m.V + kNeRows - 1) / kNeRows;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int P = m.P;
    {
        // the three tables' first rounds read together (clamped indices; the
        // values past a table's end are not stored), the rest after
        const int n1 = 8 * m.L, n2 = 6 * P, n3 = 4 * m.L;
        const int q2 = min(tid, n2 - 1);
        const float t1 = ldg(dq + min(tid, n1 - 1));
        const float t2 = ldg(xi + 8 * (q2 / 6) + (q2 % 6));
        const uint32_t t3 = ldg(anc + min(tid, n3 - 1));
        if (tid < n1) sdq[tid] = t1;
        if (tid < n2) sxi[tid] = t2;
        if (tid < n3) sanc[tid] = t3;
        for (int q = tid + kNeThreads; q < n1; q += kNeThreads) sdq[q] = dq[q];
        for (int q = tid + kNeThreads; q < n2; q += kNeThreads) sxi[q] = xi[8 * (q / 6) + (q % 6)];
        for (int q = tid + kNeThreads; q < n3; q += kNeThreads) sanc[q] = anc[q];
    }

    const int nb = PP >> 4;
    const int nbt = nb * (nb + 1) / 2;
    f4 acc[kNeBlocks];
#pragma unroll
    for (int q = 0; q < kNeBlocks; ++q) acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    __syncthreads();

    for (int chunk = wg; chunk < nchunks; chunk += S.negrid) {
        __syncthreads();  // the previous chunk's tile and counts are consumed
        // 1. compact the observed vertices of this chunk (every read of a
        //    vertex's row issued before the compaction)
        bool obs = false;
        int i = chunk * kNeRows + tid;
        VertexIn in;
        if (tid < kNeRows && i < m.V) {
            vertex_load(m, i, v, n, phi, a, in);
            obs = in.cnt > 0u && (in.nx * in.nx + in.ny * in.ny + in.nz * in.nz) > 0.0f;
        }
        unsigned long long bal = __ballot(obs);
        // the columns of J the chunk's rows can touch: the union of their
        // links' ancestor masks (the other columns are zero in the tile)
        uint32_t mk[4] = {0u, 0u, 0u, 0u};
        if (obs) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int l = (in.links >> (8 * k)) & 0xFF;
                if (l != 0xFF) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) mk[w] |= sanc[4 * l + w];
                }
            }
        }
#pragma unroll
        for (int w = 0; w < 4; ++w)
            for (int o = 32; o > 0; o >>= 1) mk[w] |= (uint32_t)__shfl_xor((int)mk[w], o);
        if (lane == 0 && wid < 2) {
            scount[wid] = __popcll(bal);
#pragma unroll
            for (int w = 0; w < 4; ++w) smask[4 * wid + w] = mk[w];
        }
        __syncthreads();
        const int nrows = scount[0] + scount[1];
        uint32_t um[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) um[w] = smask[w] | smask[4 + w];
        if (obs) {
            int row = __popcll(bal & ((1ull << lane) - 1ull)) + (wid == 1 ? scount[0] : 0);
            float r;
            vertex_terms(sdq, in, &sG[row * kGStride], r, S.blend == kBlendLinear);
            sr[row] = r;
            slink[row] = in.links;
        }
        __syncthreads();
        if (nrows == 0) continue;
        const int kstep = MODE == 0 ? 16 : 32;
        const int npad = (nrows + kstep - 1) / kstep * kstep;

        // 2. rows of [J r] into the [col][row] tile.  Thread = (row, group of
        //    columns): a row's per-influence 6-vectors and its links'
        //    ancestor masks stay in registers while it walks its columns.
        {
            const int R = npad <= 64 ? 64 : 128;
            const int row = tid & (R - 1), ng = kNeThreads / R;
            const int cpg = (PP + ng - 1) / ng;
            const int c0 = (tid / R) * cpg, c1 = min(PP, c0 + cpg);
            if (row < npad && c0 < c1) {
                const bool have = row < nrows;
                const uint32_t lk = have ? slink[row] : 0xFFFFFFFFu;
                float g[24];
#pragma unroll
                for (int q = 0; q < 24; ++q) g[q] = have ? sG[row * kGStride + q] : 0.0f;
                const float rr = have ? sr[row] : 0.0f;
                auto put = [&](int col, float val) {
                    const int at = col * kJTStride + row;
                    if (MODE == 0) {
                        sJT[at] = val;
                    } else {
                        __bf16 h = (__bf16)val;
                        float rem = val - (float)h;
                        __bf16 m = (__bf16)rem;
                        plane0[at] = h;
                        plane1[at] = m;
                        if (MODE == 2) plane2[at] = (__bf16)(rem - (float)m);
                    }
                };
                int lb[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int l = (lk >> (8 * k)) & 0xFF;
                    lb[k] = l == 0xFF ? -1 : 4 * l;
                }
                // the columns of J in runs of up to 32 that share a word of the
                // links' ancestor masks (shifted one bit per column); the next
                // column's twists are read before this column is stored, so
                // the read overlaps this column's arithmetic
                const int cj = min(c1, P);
                float xn[6];
                if (c0 < cj) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) xn[e] = sxi[6 * c0 + e];
                }
                for (int col = c0; col < cj;) {
                    const int run_end = min(cj, (col & ~31) + 32);
                    uint32_t cur[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) cur[k] = lb[k] < 0 ? 0u : sanc[lb[k] + (col >> 5)] >> (col & 31);
                    const uint32_t uw = um[col >> 5];
                    for (; col < run_end; ++col) {
                        const float x0 = xn[0], x1 = xn[1], x2 = xn[2], x3 = xn[3], x4 = xn[4], x5 = xn[5];
                        const int cn = min(col + 1, cj - 1);
#pragma unroll
                        for (int e = 0; e < 6; ++e) xn[e] = sxi[6 * cn + e];
                        float val = 0.0f;
                        if ((uw >> (col & 31)) & 1u) {   // a column some row of the chunk touches
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const float* gk = g + 6 * k;
                                const float dt = gk[0] * x0 + gk[1] * x1 + gk[2] * x2 + gk[3] * x3 + gk[4] * x4 +
                                                 gk[5] * x5;
                                const float nv = val - dt;
                                val = (cur[k] & 1u) ? nv : val;
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k) cur[k] >>= 1;
                        put(col, val);
                    }
                }
                // the residual column, then the padding
                for (int col = max(c0, P); col < c1; ++col) put(col, col == P ? rr : 0.0f);
            }
        }
        __syncthreads();

        // 3. Gram blocks (I <= J) owned by this wave
#pragma unroll
        for (int q = 0; q < kNeBlocks; ++q) {
            const int idx = wid + kNeWaves * q;
            int I = 0, J = 0;
            if (idx < nbt) block_of(idx, nb, I, J);
            // a block of columns no row touches (and without the residual)
            // is zero in the tile: its products are skipped
            auto blk_used = [&](int K) { return ((um[K >> 1] >> ((K & 1) * 16)) & 0xFFFFu) != 0u || (P >> 4) == K; };
            if (idx < nbt && blk_used(I) && blk_used(J)) {
                const int ca = (I * 16 + (lane & 15)) * kJTStride;
                const int cb = (J * 16 + (lane & 15)) * kJTStride;
                if (MODE == 0) {
                    for (int k0 = 0; k0 < npad; k0 += 16) {
                        const int ro = k0 + 4 * (lane >> 4);
                        f4 av = *reinterpret_cast<const f4*>(&sJT[ca + ro]);
                        f4 bv = *reinterpret_cast<const f4*>(&sJT[cb + ro]);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc[q], 0, 0, 0);
                    }
                } else {
                    for (int k0 = 0; k0 < npad; k0 += 32) {
                        const int ro = k0 + 8 * (lane >> 4);
                        bf8 ah = *reinterpret_cast<const bf8*>(&plane0[ca + ro]);
                        bf8 am = *reinterpret_cast<const bf8*>(&plane1[ca + ro]);
                        bf8 bh = *reinterpret_cast<const bf8*>(&plane0[cb + ro]);
                        bf8 bm = *reinterpret_cast<const bf8*>(&plane1[cb + ro]);
                        // smallest products first
                        if (MODE == 2) {
                            bf8 al = *reinterpret_cast<const bf8*>(&plane2[ca + ro]);
                            bf8 bl = *reinterpret_cast<const bf8*>(&plane2[cb + ro]);
                            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[q], 0, 0, 0);
                            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[q], 0, 0, 0);
                            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc[q], 0, 0, 0);
                        }
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[q], 0, 0, 0);
                    }
                }
            }
        }
    }

    // 4. this workgroup's partial Gram (upper blocks only)
    float* out = S.partials + (size_t)wg * PP * PP;
#pragma unroll
    for (int q = 0; q < kNeBlocks; ++q) {
        const int idx = wid + kNeWaves * q;
        if (idx < nbt) {
            int I, J;
            block_of(idx, nb, I, J);
            const int j = J * 16 + (lane & 15);
            const int i0 = I * 16 + 4 * (lane >> 4);
            out[(i0 + 0) * PP + j] = acc[q][0];
            out[(i0 + 1) * PP + j] = acc[q][1];
            out[(i0 + 2) * PP + j] = acc[q][2];
            out[(i0 + 3) * PP + j] = acc[q][3];
        }
    }
}

// one chunk per workgroup up to 512 workgroups (two per CU fit with the LDS
// of a 75-joint body); larger meshes loop over chunks
int ne_grid(int V) {
    int nchunks = (V + kNeRows - 1) / kNeRows;
    return nchunks < 512 ? nchunks : 512;
}

constexpr size_t kSmallLds = 64 * 1024;

bool prepare_normal_eq() {
    bool ok = true;
    ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_normal_eq<0, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ne_lds_bytes<0>(kPPMax, kMaxLinks + 1)) == hipSuccess && ok;
    ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_normal_eq<1, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ne_lds_bytes<1>(kPPMax, kMaxLinks + 1)) == hipSuccess && ok;
    ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_normal_eq<2, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ne_lds_bytes<2>(kPPMax, kMaxLinks + 1)) == hipSuccess && ok;
    return ok;
}

template <int MODE>
void launch_normal_eq_t(const Launch& L, int vsel, int pn) {
    const dim3 g(L.grid[KK_NE]);
    const int pp = L.ne_pp, lm = L.ne_l;
    const size_t bytes = ne_lds_bytes<MODE>(pp, lm);
    if (bytes <= kSmallLds)
        launch_kernel(L, true, true, k_normal_eq<MODE, false>, g, dim3(kNeThreads), bytes, L.B.slots, L.B.pre, L.B.n, vsel, pn, pp, lm);
    else
        launch_kernel(L, true, true, k_normal_eq<MODE, true>, g, dim3(kNeThreads), bytes, L.B.slots, L.B.pre, L.B.n, vsel, pn, pp, lm);
}

void launch_normal_eq(const Launch& L, int gram_mode, int vsel, int pn) {
    if (gram_mode == 0) launch_normal_eq_t<0>(L, vsel, pn);
    else if (gram_mode == 1) launch_normal_eq_t<1>(L, vsel, pn);
    else launch_normal_eq_t<2>(L, vsel, pn);
}

// Sum of the partial Gram matrices in workgroup order, in float64; writes the
// full symmetric matrix (the upper triangle is summed and mirrored, so the
// result is exactly symmetric).  A workgroup handles 32 elements of one
// 16x16 block; each element's partials are split into kRedGroups contiguous
// groups summed by as many threads (a few rounds of eight loads each), and
// the group sums are added in group order.
constexpr int kRedGroups = 16;
__global__ void __launch_bounds__(32 * kRedGroups) k_gram_reduce(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn) {
    const Batch B{bs, bp, bn};
    __shared__ double part[kRedGroups][32];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_REDUCE, blockIdx.x, local)];
    const int PP = S.PP, nparts = S.negrid;
    const float* __restrict__ partials = S.partials;
    double* __restrict__ gram = S.gram;
    const int nb = PP >> 4;
    const int blk = local >> 3;               // 8 workgroups per 16x16 block
    const int el = (local & 7) * 32 + (threadIdx.x & 31);
    const int grp = threadIdx.x >> 5;
    int I, J;
    block_of(blk, nb, I, J);
    const int i = I * 16 + (el >> 4), j = J * 16 + (el & 15);
    // the tree-form pose solve takes this element (damped, frozen) in its front image
    // (its reads unconditional at clamped indices, issued with the partials'
    // below: a read under a condition is waited for inside it)
    const int* __restrict__ gfm = S.tree.gfmap;
    const int P = S.m.P;
    int fe = -1;
    double prior_i = 0.0, theta_i = 0.0;
    int act_i = 0, act_j = 0;
    if (gfm) {   // the same for the whole workgroup
        const int ic = min(i, P - 1), jc = min(j, P - 1);
        const int f0 = gfm[i * PP + j];
        const double pr = S.jt->prior[ic], th = S.theta[ic];
        const int ai = S.jt->active[ic], aj = S.jt->active[jc];
        fe = (grp == 0 && i <= j) ? f0 : -1;
        if (fe >= 0) {
            prior_i = pr;
            act_i = ai;
            act_j = j < P ? aj : 1;
            theta_i = th;
        }
    }
    const size_t stride = (size_t)PP * PP;
    const int per = (nparts + kRedGroups - 1) / kRedGroups;
    const int q0 = grp * per, q1 = min(nparts, q0 + per);
    const float* p = partials + (size_t)i * PP + j;
    double s = 0.0;
    int q = q0;
    for (; q + 8 <= q1; q += 8) {
        float a[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) a[t] = p[(size_t)(q + t) * stride];
#pragma unroll
        for (int t = 0; t < 8; ++t) s += (double)a[t];
    }
    for (; q < q1; ++q) s += (double)p[(size_t)q * stride];
    part[grp][threadIdx.x & 31] = s;
    __syncthreads();
    if (grp == 0 && i <= j) {
        double tot = 0.0;
        for (int g = 0; g < kRedGroups; ++g) tot += part[g][threadIdx.x & 31];
        gram[i * PP + j] = tot;
        gram[j * PP + i] = tot;
        if (fe >= 0) {
            // as the dense solve sets up its matrix: a joint with no weight
            // (zero diagonal: its whole row is zero) or masked inactive is
            // frozen to an identity row with a zero right-hand side
            double v;
            if (j == P) v = act_i ? tot + prior_i * theta_i : 0.0;
            else if (i == j) v = (tot + prior_i == 0.0 || !act_i) ? 1.0 : (tot + prior_i) * (1.0 + (double)S.lambda_k);
            else v = (act_i && act_j) ? tot : 0.0;
            S.tree.fimg[fe] = v;
        }
    }
}

void launch_gram_reduce(const Launch& L) {
    launch_kernel(L, true, true, k_gram_reduce, dim3(L.grid[KK_REDUCE]), dim3(32 * kRedGroups), 0, L.B.slots, L.B.pre, L.B.n);
}

}  // namespace trk
