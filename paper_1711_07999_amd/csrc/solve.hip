// Pose step (Section 4.2) and per-vertex offset step (Section 4.3).
#include "common.h"
#include "dq.h"
#include "fk.h"

namespace trk {

// ---------------------------------------------------------------------------
// Damped least squares (Marquardt): (A + lambda_k diag(A)) x = b with
// A = J^T J + (lambda_s S)^2 and b = J^T r + (lambda_s S)^2 Theta, solved by
// Cholesky in one workgroup; Theta <- Theta - x.  Parameters with A_kk == 0
// (no observed vertex moves them) or marked inactive are frozen (x_k = 0).
// A failed factorisation leaves Theta unchanged and flags the frame.  The
// same workgroup then runs forward kinematics at the new pose.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_pose_solve(const JointTable* __restrict__ jt, int PP,
                                                    const double* __restrict__ gram, float lambda_k,
                                                    double* __restrict__ theta, double* __restrict__ step,
                                                    DevStats* st, int iter, float* dq, float* xi) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int P = jt->P;
    T* M = reinterpret_cast<T*>(smem);       // [P][P] row-major, lower triangle used
    T* y = M + P * P;                         // [P]
    __shared__ int frozen[kMaxJoints + 1];
    __shared__ int fail;
    const int tid = threadIdx.x;
    if (tid == 0) fail = 0;
    for (int k = tid; k < P; k += 256) {
        double akk = gram[k * PP + k] + jt->prior[k];
        frozen[k] = (akk == 0.0) || !jt->active[k];
    }
    __syncthreads();
    for (int e = tid; e < P * P; e += 256) {
        int k = e / P, q = e - k * P;
        double a = gram[k * PP + q] + (k == q ? jt->prior[k] : 0.0);
        T val;
        if (k == q) val = frozen[k] ? T(1) : T(a * (1.0 + (double)lambda_k));
        else val = (frozen[k] || frozen[q]) ? T(0) : T(a);
        M[e] = val;
    }
    for (int k = tid; k < P; k += 256)
        y[k] = frozen[k] ? T(0) : T(gram[k * PP + P] + jt->prior[k] * theta[k]);
    __syncthreads();
    // right-looking Cholesky, M = L L^T in the lower triangle
    for (int j = 0; j < P; ++j) {
        if (tid == 0) {
            T d = M[j * P + j];
            if (!(d > T(0))) fail = 1;
            else M[j * P + j] = sqrt(d);
        }
        __syncthreads();
        if (fail) break;
        const T djj = M[j * P + j];
        for (int i = j + 1 + tid; i < P; i += 256) M[i * P + j] /= djj;
        __syncthreads();
        const int nrem = P - j - 1;
        for (int e = tid; e < nrem * nrem; e += 256) {
            int ii = e / nrem, kk = e - ii * nrem;
            if (kk <= ii) {
                int i = j + 1 + ii, k = j + 1 + kk;
                M[i * P + k] -= M[i * P + j] * M[k * P + j];
            }
        }
        __syncthreads();
    }
    if (!fail) {
        // L z = b, then L^T x = z
        for (int j = 0; j < P; ++j) {
            if (tid == 0) y[j] /= M[j * P + j];
            __syncthreads();
            for (int i = j + 1 + tid; i < P; i += 256) y[i] -= M[i * P + j] * y[j];
            __syncthreads();
        }
        for (int j = P - 1; j >= 0; --j) {
            if (tid == 0) y[j] /= M[j * P + j];
            __syncthreads();
            for (int i = tid; i < j; i += 256) y[i] -= M[j * P + i] * y[j];
            __syncthreads();
        }
        __shared__ double nrm[256];
        double part = 0.0;
        for (int k = tid; k < P; k += 256) {
            double x = frozen[k] ? 0.0 : (double)y[k];
            step[k] = x;
            theta[k] -= x;
            part += x * x;
        }
        nrm[tid] = part;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int q = 0; q < 256; ++q) s += nrm[q];
            st->step_norm[iter] = (float)sqrt(s);
            st->energy[iter] = (float)gram[P * PP + P];
        }
    } else if (tid == 0) {
        st->status = -4;
        st->energy[iter] = (float)gram[P * PP + P];
        st->step_norm[iter] = 0.0f;
    }
    __syncthreads();
    fk_block(jt, theta, dq, xi);
}

void launch_pose_solve(hipStream_t s, const JointTable* jt, int PP, const double* gram, float lambda_k,
                       int fp64, double* theta, double* step, DevStats* st, int iter, float* dq, float* xi) {
    int P = PP;  // upper bound on P for the LDS size
    if (fp64) {
        size_t sh = (size_t)(P * P + P) * sizeof(double);
        hipLaunchKernelGGL(k_pose_solve<double>, dim3(1), dim3(256), sh, s, jt, PP, gram, lambda_k, theta, step,
                           st, iter, dq, xi);
    } else {
        size_t sh = (size_t)(P * P + P) * sizeof(float);
        hipLaunchKernelGGL(k_pose_solve<float>, dim3(1), dim3(256), sh, s, jt, PP, gram, lambda_k, theta, step,
                           st, iter, dq, xi);
    }
}

// ---------------------------------------------------------------------------
// Per-vertex offset step (reading of Eq. 9 as a sum of squared residuals with
// the neighbours held fixed, the independence approximation of Section 4.3):
//   u_i = -R_i^T n_i (0 if unobserved),  r_i = n_i . delta_i,
//   g_i = u_i r_i + lam_phi phi_i + lam_N sum_n (phi_i - phi_n)
//         + lam_T (phi_i - phi_i^prev),
//   A_i = u_i u_i^T + (lam_phi + lam_N |N(i)| + lam_T) I,
//   (A_i + lam_w diag A_i) x_i = g_i,  phi_i <- phi_i - x_i,
// with delta_i = (sum of p - v at association) / c_i + (v_old - v_new) after
// a pose step.  One vertex per lane; the 3x3 solve in float32 or float64.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void solve3(const T M[9], const T g[3], T x[3]) {
    T c00 = M[4] * M[8] - M[5] * M[7], c01 = M[5] * M[6] - M[3] * M[8], c02 = M[3] * M[7] - M[4] * M[6];
    T det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    if (!(fabs(det) > T(0))) { x[0] = x[1] = x[2] = T(0); return; }
    T i0[3] = {c00, M[2] * M[7] - M[1] * M[8], M[1] * M[5] - M[2] * M[4]};
    T i1[3] = {c01, M[0] * M[8] - M[2] * M[6], M[2] * M[3] - M[0] * M[5]};
    T i2[3] = {c02, M[1] * M[6] - M[0] * M[7], M[0] * M[4] - M[1] * M[3]};
    x[0] = (i0[0] * g[0] + i0[1] * g[1] + i0[2] * g[2]) / det;
    x[1] = (i1[0] * g[0] + i1[1] * g[1] + i1[2] * g[2]) / det;
    x[2] = (i2[0] * g[0] + i2[1] * g[1] + i2[2] * g[2]) / det;
}

template <class T>
__global__ void __launch_bounds__(256) k_shape(DevModel m, const float* __restrict__ dq, CVec3Buf v_old,
                                               CVec3Buf v_new, CVec3Buf n, Accum a, CVec3Buf phi,
                                               CVec3Buf phi_prev, Vec3Buf phi_out, float lphi, float lnbr,
                                               float lt, float lw) {
    __shared__ float sdq[8 * (kMaxLinks + 1)];
    for (int q = threadIdx.x; q < 8 * m.L; q += blockDim.x) sdq[q] = dq[q];
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.V) return;
    const T px = phi.x[i], py = phi.y[i], pz = phi.z[i];
    T u[3] = {T(0), T(0), T(0)};
    T r = T(0);
    const uint32_t c = a.cnt[i];
    const float nx = n.x[i], ny = n.y[i], nz = n.z[i];
    if (c > 0u && (nx * nx + ny * ny + nz * nz) > 0.0f) {
        float H[8];
        dq_blend(sdq, m.w[i], m.links[i], H);
        T w = H[0], x = H[1], y = H[2], z = H[3];
        T s = T(2) / (w * w + x * x + y * y + z * z);
        T R[9] = {T(1) - s * (y * y + z * z), s * (x * y - w * z), s * (x * z + w * y),
                  s * (x * y + w * z), T(1) - s * (x * x + z * z), s * (y * z - w * x),
                  s * (x * z - w * y), s * (y * z + w * x), T(1) - s * (x * x + y * y)};
        for (int q = 0; q < 3; ++q) u[q] = -(R[q] * nx + R[3 + q] * ny + R[6 + q] * nz);
        const T inv = T(1) / ((T)c * T(4294967296.0));
        T dx = (T)a.sx[i] * inv + ((T)v_old.x[i] - (T)v_new.x[i]);
        T dy = (T)a.sy[i] * inv + ((T)v_old.y[i] - (T)v_new.y[i]);
        T dz = (T)a.sz[i] * inv + ((T)v_old.z[i] - (T)v_new.z[i]);
        r = (T)nx * dx + (T)ny * dy + (T)nz * dz;
    }
    T alpha = (T)lphi + (T)lt;
    T g[3] = {u[0] * r + (T)lphi * px + (T)lt * (px - (T)phi_prev.x[i]),
              u[1] * r + (T)lphi * py + (T)lt * (py - (T)phi_prev.y[i]),
              u[2] * r + (T)lphi * pz + (T)lt * (pz - (T)phi_prev.z[i])};
    const int4 nb = m.nbr[i];
    const int nbs[4] = {nb.x, nb.y, nb.z, nb.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int j = nbs[q];
        if (j < 0) continue;
        alpha += (T)lnbr;
        g[0] += (T)lnbr * (px - (T)phi.x[j]);
        g[1] += (T)lnbr * (py - (T)phi.y[j]);
        g[2] += (T)lnbr * (pz - (T)phi.z[j]);
    }
    T M[9];
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) M[3 * p + q] = u[p] * u[q] + (p == q ? alpha : T(0));
    for (int p = 0; p < 3; ++p) M[4 * p] *= (T(1) + (T)lw);
    T xs[3];
    solve3(M, g, xs);
    phi_out.x[i] = (float)(px - xs[0]);
    phi_out.y[i] = (float)(py - xs[1]);
    phi_out.z[i] = (float)(pz - xs[2]);
}

void launch_shape(hipStream_t s, const DevModel& m, const float* dq, CVec3Buf v_old, CVec3Buf v_new,
                  CVec3Buf n, const Accum& a, CVec3Buf phi, CVec3Buf phi_prev, Vec3Buf phi_out,
                  float lphi, float lnbr, float lt, float lw, int fp64) {
    int grid = (m.V + 255) / 256;
    if (fp64)
        hipLaunchKernelGGL(k_shape<double>, dim3(grid), dim3(256), 0, s, m, dq, v_old, v_new, n, a, phi, phi_prev,
                           phi_out, lphi, lnbr, lt, lw);
    else
        hipLaunchKernelGGL(k_shape<float>, dim3(grid), dim3(256), 0, s, m, dq, v_old, v_new, n, a, phi, phi_prev,
                           phi_out, lphi, lnbr, lt, lw);
}

}  // namespace trk
