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
                                              Vec3Buf v) {
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
    v.x[i] = ox; v.y[i] = oy; v.z[i] = oz;
}

void launch_skin(hipStream_t s, const DevModel& m, const float* dq, CVec3Buf phi, Vec3Buf v) {
    int grid = (m.V + 255) / 256;
    hipLaunchKernelGGL(k_skin, dim3(grid), dim3(256), 0, s, m, dq, phi, v);
}

// ---------------------------------------------------------------------------
// Vertex normals: the sum over incident faces of their doubled-area normal
// vectors, normalised (zero if the sum vanishes).  Each vertex gathers its own
// fan (no atomics, deterministic).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_normals(DevModel m, CVec3Buf v, Vec3Buf n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.V) return;
    float px = v.x[i], py = v.y[i], pz = v.z[i];
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    uint32_t e0 = m.fan_off[i], e1 = m.fan_off[i + 1];
    for (uint32_t e = e0; e < e1; ++e) {
        int2 bc = m.fan[e];
        float ax = v.x[bc.x] - px, ay = v.y[bc.x] - py, az = v.z[bc.x] - pz;
        float bx = v.x[bc.y] - px, by = v.y[bc.y] - py, bz = v.z[bc.y] - pz;
        sx += ay * bz - az * by;
        sy += az * bx - ax * bz;
        sz += ax * by - ay * bx;
    }
    float l = sqrtf(sx * sx + sy * sy + sz * sz);
    float inv = l > 0.0f ? 1.0f / l : 0.0f;
    n.x[i] = sx * inv; n.y[i] = sy * inv; n.z[i] = sz * inv;
}

void launch_normals(hipStream_t s, const DevModel& m, CVec3Buf v, Vec3Buf n) {
    int grid = (m.V + 255) / 256;
    hipLaunchKernelGGL(k_normals, dim3(grid), dim3(256), 0, s, m, v, n);
}

__global__ void k_copy3(int V, CVec3Buf src, Vec3Buf dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    dst.x[i] = src.x[i]; dst.y[i] = src.y[i]; dst.z[i] = src.z[i];
}

void launch_copy3(hipStream_t s, int V, CVec3Buf src, Vec3Buf dst) {
    hipLaunchKernelGGL(k_copy3, dim3((V + 255) / 256), dim3(256), 0, s, V, src, dst);
}

}  // namespace trk
