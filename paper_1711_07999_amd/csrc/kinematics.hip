// Forward kinematics, blend skinning and vertex normals (Sections 3.1, 3.2),
// and the per-frame bookkeeping kernels, over a batch of slots.
#include "common.h"
#include "dq.h"
#include "fk.h"
#include "surface.h"

namespace trk {

// ---------------------------------------------------------------------------
// table upload: the host writes the slot table into pinned memory and this
// first kernel of a launch copies it to device memory (no copy engine call)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_stage(const uint4* __restrict__ src, uint4* __restrict__ dst, int n16,
                                               const int* __restrict__ psrc, int* __restrict__ pdst, int npre) {
    for (int i = threadIdx.x; i < n16; i += 256) dst[i] = src[i];
    for (int i = threadIdx.x; i < npre; i += 256) pdst[i] = psrc[i];
}

void launch_stage(hipStream_t s, const Slot* src, Slot* dst, int n, const int* psrc, int* pdst, int npre) {
    const int n16 = (int)(sizeof(Slot) / 16) * n;
    hipLaunchKernelGGL(k_stage, dim3(1), dim3(256), 0, s, reinterpret_cast<const uint4*>(src),
                       reinterpret_cast<uint4*>(dst), n16, psrc, pdst, npre);
}

// ---------------------------------------------------------------------------
// frame start: keep the pose for a rollback, clear the status flag and (when
// the slot asks for it) redo forward kinematics at the current pose
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) k_frame_begin(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_ONE, blockIdx.x, local)];
    if (!(S.flags & kSlotBeginFrame)) return;
    __shared__ FkScratch ws;
    const int P = S.m.P;
    for (int k = threadIdx.x; k < P; k += blockDim.x) S.theta_backup[k] = S.theta[k];
    if (threadIdx.x == 0) S.st->status = 0;
    if (S.flags & kSlotRefreshPose) fk_block(S.jt, S.m.P, S.m.L, S.theta, S.dq, S.xi, ws);
}

void launch_frame_begin(const Launch& L) {
    launch_kernel(L, true, true, k_frame_begin, dim3(L.grid[KK_ONE]), dim3(128), 0, L.B.slots, L.B.pre, L.B.n);
}

__global__ void __launch_bounds__(128) k_fk(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_ONE, blockIdx.x, local)];
    __shared__ FkScratch ws;
    fk_block(S.jt, S.m.P, S.m.L, S.theta, S.dq, S.xi, ws);
}

void launch_fk(const Launch& L) {
    launch_kernel(L, true, true, k_fk, dim3(L.grid[KK_ONE]), dim3(128), 0, L.B.slots, L.B.pre, L.B.n);
}

// ---------------------------------------------------------------------------
// Skinning (Eq. 3 and 5): v_i = T(sum_j w_ij H_{j,Delta}, v0_i + phi_i), one
// vertex per lane, link offsets staged in LDS, coalesced SoA streams.  The
// vertex can also be counted into the bucket index of the next association
// (or only counted, to lay out the index), and the per-vertex accumulators
// of the last association cleared, so that neither needs a launch of its own.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_skin(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vsel, int pn, int which, int count, int bsel, int count_only,
                                              int clear_acc) {
    const Batch B{bs, bp, bn};
    __shared__ float sdq[8 * (kMaxLinks + 1)];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_VERT64, blockIdx.x, local)];
    if (!selected(S, which)) return;
    const DevModel& m = S.m;
    const bool counted = selected(S, count);
    const CountRefs cr = count_refs(S, bsel);
    const int i = local * blockDim.x + threadIdx.x;
    const int ii = i < m.V ? i : 0;   // the vertex's own loads go out before the table copy
    const Vec3Buf phi = S.phi[phi_index(S, pn)];
    const float4 w = m.w[ii];
    const uint32_t lk = m.links[ii];
    float x = m.rx[ii] + phi.x[ii], y = m.ry[ii] + phi.y[ii], z = m.rz[ii] + phi.z[ii];
    copy_to_lds(sdq, S.dq, 8 * m.L);
    __syncthreads();
    const bool live = i < m.V;   // lanes past the end skin vertex 0 and store nothing
    float4* __restrict__ v = S.verts[S.v_cur ^ vsel];
    float ox, oy, oz;
    if (S.blend == kBlendLinear) {
        lbs_apply(sdq, w, lk, x, y, z, ox, oy, oz);
    } else {
        float H[8];
        dq_blend(sdq, w, lk, H);
        dq_apply(H, x, y, z, ox, oy, oz);
    }
    const float4 p = make_float4(ox, oy, oz, 0.0f);
    if (live) stg(v + i, p);
    if (counted) count_vertex(cr, i, p, live, count_only != 0);   // the whole wave
    if (live && clear_acc) {
        S.a.cnt[i] = 0u;
        S.a.sx[i] = 0; S.a.sy[i] = 0; S.a.sz[i] = 0;
    }
}

void launch_skin(const Launch& L, int vsel, int pn, int which, int count, int bsel, int count_only, int clear_acc) {
    // one wave per workgroup: the vertices spread over every compute unit
    launch_kernel(L, true, true, k_skin, dim3(L.grid[KK_VERT64]), dim3(64), 0, L.B.slots, L.B.pre, L.B.n, vsel, pn, which, count, bsel,
                  count_only, clear_acc);
}

// Vertex normals (one lane per vertex; see vertex_normal)
__global__ void __launch_bounds__(256) k_normals(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vsel) {
    const Batch B{bs, bp, bn};
    int local;
    const Slot& S = B.slots[slot_of(B, KK_VERT, blockIdx.x, local)];
    const int i = local * blockDim.x + threadIdx.x;
    const bool live = i < S.m.V;
    float nx, ny, nz;
    vertex_normal(S.m, S.verts[S.v_cur ^ vsel], i, live, nx, ny, nz);   // the whole wave
    if (live) { S.normals.x[i] = nx; S.normals.y[i] = ny; S.normals.z[i] = nz; }
}

void launch_normals(const Launch& L, int vsel) {
    launch_kernel(L, true, true, k_normals, dim3(L.grid[KK_VERT]), dim3(256), 0, L.B.slots, L.B.pre, L.B.n, vsel);
}

// ---------------------------------------------------------------------------
// frame end: the health check of the frame (solver failure, no valid pixel,
// no matched pixel, non-finite pose or energy); on failure the pose is rolled
// back to the frame's start (the offsets are rolled back by the host, which
// keeps the frame-start offset buffer untouched).  The per-tile counts of the
// last association are summed into the slot's summary.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_frame_end(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int first_pose, int last_pose) {
    const Batch B{bs, bp, bn};
    __shared__ int s_sum[3][4];
    __shared__ int s_bad;
    int local;
    const Slot& S = B.slots[slot_of(B, KK_ONE, blockIdx.x, local)];
    if (!(S.flags & kSlotEndFrame)) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ntiles = S.c.tiles_x * S.c.tiles_y;
    int nv = 0, na = 0, no = 0;
    for (int t = tid; t < ntiles; t += 256 * 20) {   // one round of loads up to 5120 tiles
        int4 q[20];
#pragma unroll
        for (int j = 0; j < 20; ++j) q[j] = S.b.bstat[min(t + 256 * j, ntiles - 1)];   // past the end: not added
#pragma unroll
        for (int j = 0; j < 20; ++j)
            if (t + 256 * j < ntiles) { nv += q[j].x; na += q[j].y; no += q[j].z; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        nv += __shfl_xor(nv, o);
        na += __shfl_xor(na, o);
        no += __shfl_xor(no, o);
    }
    if (lane == 0) { s_sum[0][wid] = nv; s_sum[1][wid] = na; s_sum[2][wid] = no; }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int k = tid; k < S.m.P; k += 256)
        if (!isfinite(S.theta[k])) s_bad = 1;
    __syncthreads();
    if (tid == 0) {
        nv = na = no = 0;
        for (int q = 0; q < 4; ++q) { nv += s_sum[0][q]; na += s_sum[1][q]; no += s_sum[2][q]; }
        DevStats* st = S.st;
        DevSummary& out = *S.summary;
        out.n_valid_px = nv;
        out.n_assoc_px = na;
        out.n_obs_verts = no;
        out.energy_first = first_pose >= 0 ? st->energy[first_pose] : 0.0f;
        out.energy_last = last_pose >= 0 ? st->energy[last_pose] : 0.0f;
        out.step_norm_last = last_pose >= 0 ? st->step_norm[last_pose] : 0.0f;
        int status = 0, why = 0;
        if (st->status == -4) { status = -4; why = 1; }
        else if (st->status == kStatusBucketOverflow) { status = -5; why = 6; }
        else if (nv == 0) { status = -5; why = 2; }
        else if (na == 0) { status = -5; why = 3; }
        else if (s_bad) { status = -5; why = 4; }
        else if (!isfinite(out.energy_last)) { status = -5; why = 5; }
        out.status = status;
        out.reason = why;
        s_bad = status != 0;
    }
    __syncthreads();
    if (s_bad)
        for (int k = tid; k < S.m.P; k += 256) S.theta[k] = S.theta_backup[k];
}

void launch_frame_end(const Launch& L, int first_pose, int last_pose) {
    launch_kernel(L, true, true, k_frame_end, dim3(L.grid[KK_ONE]), dim3(256), 0, L.B.slots, L.B.pre, L.B.n, first_pose, last_pose);
}

}  // namespace trk
