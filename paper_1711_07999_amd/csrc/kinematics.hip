// Forward kinematics, blend skinning and vertex normals (Sections 3.1, 3.2).
#include "common.h"
#include "dq.h"
#include "fk.h"

namespace trk {

__global__ void __launch_bounds__(128) k_fk(const JointTable* jt, const double* theta, float* dq, float* xi) {
    fk_block(jt, theta, dq, xi);
}

void launch_fk(hipStream_t s, const JointTable* jt, const double* theta, float* dq, float* xi) {
    hipLaunchKernelGGL(k_fk, dim3(1), dim3(128), 0, s, jt, theta, dq, xi);
}

// ---------------------------------------------------------------------------
// Skinning (Eq. 3 and 5): v_i = T(sum_j w_ij H_{j,Delta}, v0_i + phi_i), one
// vertex per lane, link offsets staged in LDS, coalesced SoA streams.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_skin(DevModel m, const float* __restrict__ dq, CVec3Buf phi,
                                              float4* __restrict__ v) {
    __shared__ float sdq[8 * (kMaxLinks + 1)];
    for (int q = threadIdx.x; q < 8 * m.L; q += blockDim.x) sdq[q] = dq[q];
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.V) return;
    float H[8];
    dq_blend(sdq, m.w[i], m.links[i], H);
    float x = m.rx[i] + phi.x[i], y = m.ry[i] + phi.y[i], z = m.rz[i] + phi.z[i];
    float ox, oy, oz;
    dq_apply(H, x, y, z, ox, oy, oz);
    v[i] = make_float4(ox, oy, oz, 0.0f);
}

void launch_skin(hipStream_t s, const DevModel& m, const float* dq, CVec3Buf phi, float4* v) {
    int grid = (m.V + 255) / 256;
    hipLaunchKernelGGL(k_skin, dim3(grid), dim3(256), 0, s, m, dq, phi, v);
}

// ---------------------------------------------------------------------------
// Vertex normals: the sum over incident faces of their doubled-area normal
// vectors, normalised (zero if the sum vanishes).  Each vertex gathers its own
// fan (no atomics, deterministic); four lanes share one vertex's fan and
// combine their partial sums with lane shuffles in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kNormLanes = 4;

__global__ void __launch_bounds__(256) k_normals(DevModel m, const float4* __restrict__ v, Vec3Buf n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kNormLanes, sub = t % kNormLanes;
    const bool live = i < m.V;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    if (live) {
        const float4 p = v[i];
        const uint32_t e1 = m.fan_off[i + 1];
        for (uint32_t e = m.fan_off[i] + sub; e < e1; e += kNormLanes) {
            const int2 bc = m.fan[e];
            const float4 vb = v[bc.x], vc = v[bc.y];
            float ax = vb.x - p.x, ay = vb.y - p.y, az = vb.z - p.z;
            float bx = vc.x - p.x, by = vc.y - p.y, bz = vc.z - p.z;
            sx += ay * bz - az * by;
            sy += az * bx - ax * bz;
            sz += ax * by - ay * bx;
        }
    }
    // combine the four lanes of the vertex (lanes 4i..4i+3 of one wave)
    for (int o = 1; o < kNormLanes; o <<= 1) {
        sx += __shfl_xor(sx, o);
        sy += __shfl_xor(sy, o);
        sz += __shfl_xor(sz, o);
    }
    if (!live || sub != 0) return;
    float l = sqrtf(sx * sx + sy * sy + sz * sz);
    float inv = l > 0.0f ? 1.0f / l : 0.0f;
    n.x[i] = sx * inv; n.y[i] = sy * inv; n.z[i] = sz * inv;
}

void launch_normals(hipStream_t s, const DevModel& m, const float4* v, Vec3Buf n) {
    int grid = (m.V * kNormLanes + 255) / 256;
    hipLaunchKernelGGL(k_normals, dim3(grid), dim3(256), 0, s, m, v, n);
}

__global__ void k_copy3(int V, CVec3Buf src, Vec3Buf dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    dst.x[i] = src.x[i]; dst.y[i] = src.y[i]; dst.z[i] = src.z[i];
}

// frame start: keep the pose for a rollback, clear the status flag (a kernel,
// not a memset, so that the frame can be captured in a graph)
__global__ void k_frame_begin(int P, const double* theta, double* theta_backup, DevStats* st) {
    for (int k = threadIdx.x; k < P; k += blockDim.x) theta_backup[k] = theta[k];
    if (threadIdx.x == 0) st->status = 0;
}

void launch_frame_begin(hipStream_t s, int P, const double* theta, double* theta_backup, DevStats* st) {
    hipLaunchKernelGGL(k_frame_begin, dim3(1), dim3(128), 0, s, P, theta, theta_backup, st);
}

void launch_copy3(hipStream_t s, int V, CVec3Buf src, Vec3Buf dst) {
    hipLaunchKernelGGL(k_copy3, dim3((V + 255) / 256), dim3(256), 0, s, V, src, dst);
}

}  // namespace trk
