// Pose step (Section 4.2) and per-vertex offset step (Section 4.3).
#include "common.h"
#include "dq.h"
#include "fk.h"

namespace trk {

// ---------------------------------------------------------------------------
// Damped least squares (Marquardt): (A + lambda_k diag(A)) x = b with
// A = J^T J + (lambda_s S)^2 and b = J^T r + (lambda_s S)^2 Theta, solved by
// Cholesky; Theta <- Theta - x.  Parameters with A_kk == 0 (no observed vertex
// moves them) or marked inactive are frozen (x_k = 0).  A failed
// factorisation leaves Theta unchanged and flags the frame.
//
// Blocked right-looking Cholesky in one workgroup: the matrix (padded to a
// multiple of 8 with identity rows) is split into 8x8 blocks, thread (i, j)
// of a 16x16 grid holds block (i, j) in registers.  For each 8-column panel:
// the diagonal block is factored by its thread, the blocks below are solved
// against it, and the trailing blocks take the rank-8 update, with the panel
// exchanged through LDS -- three barriers per panel.  The right-hand side is
// carried along (forward substitution) and back substitution runs panel by
// panel.  The same workgroup then runs forward kinematics at the new pose.
// ---------------------------------------------------------------------------
constexpr int kBS = 8;                    // block size
constexpr int kNBMax = (kMaxJoints + 1) / kBS;  // 16 blocks per side
constexpr int kPanelStride = kBS * kBS + 1;

template <class T>
__global__ void __launch_bounds__(256) k_pose_solve(Batch B, int iter) {
    // L blocks of the current panel column; block stride kBS*kBS + 1 keeps the
    // 16 column-block reads of a wave on distinct LDS banks
    __shared__ T s_panel[kNBMax * kPanelStride];
    __shared__ T s_y[kNBMax * kBS];           // right-hand side -> z -> x
    __shared__ T s_inv[kNBMax * kBS];         // 1 / L_jj: one division per column
    __shared__ int s_frozen[kNBMax * kBS];
    __shared__ int s_fail;
    __shared__ double s_nrm[256];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_ONE, blockIdx.x, local)];
    const JointTable* __restrict__ jt = S.jt;
    const int PP = S.PP;
    const double* __restrict__ gram = S.gram;
    const float lambda_k = S.lambda_k;
    double* __restrict__ theta = S.theta;
    double* __restrict__ step = S.step;
    DevStats* st = S.st;
    const int P = jt->P;
    const int NB = (P + kBS - 1) / kBS;
    const int tid = threadIdx.x;
    const int bi = tid >> 4, bj = tid & 15;
    const bool mine = bi < NB && bj <= bi;
    if (tid == 0) s_fail = 0;
    for (int k = tid; k < NB * kBS; k += 256) {
        int fz = 1;
        T yk = T(0);
        if (k < P) {
            const double pr = jt->prior[k];
            fz = (gram[k * PP + k] + pr == 0.0) || !jt->active[k];
            yk = fz ? T(0) : T(gram[k * PP + P] + pr * theta[k]);
        }
        s_frozen[k] = fz;
        s_y[k] = yk;
    }
    __syncthreads();
    // this thread's block of the damped, frozen and padded matrix
    T a[kBS][kBS];
#pragma unroll
    for (int r = 0; r < kBS; ++r)
#pragma unroll
        for (int c = 0; c < kBS; ++c) {
            const int i = bi * kBS + r, j = bj * kBS + c;
            T val = T(0);
            if (mine) {
                if (i == j) {
                    val = (i >= P || s_frozen[i]) ? T(1)
                                                  : T((gram[i * PP + i] + jt->prior[i]) * (1.0 + (double)lambda_k));
                } else if (i < P && j < P && !s_frozen[i] && !s_frozen[j]) {
                    val = T(gram[i * PP + j]);
                }
            }
            a[r][c] = val;
        }
    for (int p = 0; p < NB; ++p) {
        // (1) factor the diagonal block; forward-solve its part of y
        if (bi == p && bj == p) {
            bool ok = true;
#pragma unroll
            for (int j = 0; j < kBS; ++j) {
                const T d = a[j][j];
                ok = ok && (d > T(0));
                const T s = ok ? sqrt(d) : T(1);
                const T inv = T(1) / s;
                a[j][j] = s;
                s_inv[p * kBS + j] = inv;
#pragma unroll
                for (int i = j + 1; i < kBS; ++i) a[i][j] *= inv;
#pragma unroll
                for (int i = j + 1; i < kBS; ++i)
#pragma unroll
                    for (int k = j + 1; k <= i; ++k) a[i][k] -= a[i][j] * a[k][j];
            }
            T z[kBS];
#pragma unroll
            for (int r = 0; r < kBS; ++r) z[r] = s_y[p * kBS + r];
#pragma unroll
            for (int j = 0; j < kBS; ++j) {
                z[j] *= s_inv[p * kBS + j];
#pragma unroll
                for (int i = j + 1; i < kBS; ++i) z[i] -= a[i][j] * z[j];
            }
#pragma unroll
            for (int r = 0; r < kBS; ++r) {
                s_y[p * kBS + r] = z[r];
#pragma unroll
                for (int c = 0; c < kBS; ++c) s_panel[p * kPanelStride + r * kBS + c] = a[r][c];
            }
            if (!ok) s_fail = 1;
        }
        __syncthreads();
        if (s_fail) break;
        // (2) blocks below the diagonal: X L_pp^T = A_ip; update y_i
        if (bj == p && bi > p && bi < NB) {
#pragma unroll
            for (int r = 0; r < kBS; ++r) {
#pragma unroll
                for (int j = 0; j < kBS; ++j) {
                    T t = a[r][j];
#pragma unroll
                    for (int k = 0; k < j; ++k) t -= a[r][k] * s_panel[p * kPanelStride + j * kBS + k];
                    a[r][j] = t * s_inv[p * kBS + j];
                }
            }
#pragma unroll
            for (int r = 0; r < kBS; ++r) {
                T t = s_y[bi * kBS + r];
#pragma unroll
                for (int j = 0; j < kBS; ++j) {
                    t -= a[r][j] * s_y[p * kBS + j];
                    s_panel[bi * kPanelStride + r * kBS + j] = a[r][j];
                }
                s_y[bi * kBS + r] = t;
            }
        }
        __syncthreads();
        // (3) trailing update A_ij -= L_ip L_jp^T for p < j <= i
        if (mine && bj > p) {
#pragma unroll
            for (int k = 0; k < kBS; ++k) {
                T li[kBS], lj[kBS];
#pragma unroll
                for (int r = 0; r < kBS; ++r) {
                    li[r] = s_panel[bi * kPanelStride + r * kBS + k];
                    lj[r] = s_panel[bj * kPanelStride + r * kBS + k];
                }
#pragma unroll
                for (int r = 0; r < kBS; ++r)
#pragma unroll
                    for (int c = 0; c < kBS; ++c) a[r][c] -= li[r] * lj[c];
            }
        }
        __syncthreads();
    }
    const bool fail = s_fail != 0;
    if (!fail) {
        // back substitution L^T x = z, panel by panel from the last
        for (int p = NB - 1; p >= 0; --p) {
            if (bi == p && bj == p) {
                T x[kBS];
#pragma unroll
                for (int r = 0; r < kBS; ++r) x[r] = s_y[p * kBS + r];
#pragma unroll
                for (int j = kBS - 1; j >= 0; --j) {
                    x[j] *= s_inv[p * kBS + j];
#pragma unroll
                    for (int i = 0; i < j; ++i) x[i] -= a[j][i] * x[j];
                }
#pragma unroll
                for (int r = 0; r < kBS; ++r) s_y[p * kBS + r] = x[r];
            }
            __syncthreads();
            if (bi == p && bj < p) {
#pragma unroll
                for (int c = 0; c < kBS; ++c) {
                    T t = s_y[bj * kBS + c];
#pragma unroll
                    for (int r = 0; r < kBS; ++r) t -= a[r][c] * s_y[p * kBS + r];
                    s_y[bj * kBS + c] = t;
                }
            }
            __syncthreads();
        }
        double part = 0.0;
        for (int k = tid; k < P; k += 256) {
            const double x = s_frozen[k] ? 0.0 : (double)s_y[k];
            step[k] = x;
            theta[k] -= x;
            part += x * x;
        }
        s_nrm[tid] = part;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int q = 0; q < 256; ++q) s += s_nrm[q];
            st->step_norm[S.iter + iter] = (float)sqrt(s);
            st->energy[S.iter + iter] = (float)gram[P * PP + P];
        }
    } else if (tid == 0) {
        st->status = -4;
        st->energy[S.iter + iter] = (float)gram[P * PP + P];
        st->step_norm[S.iter + iter] = 0.0f;
    }
    __syncthreads();
    fk_block(jt, theta, S.dq, S.xi);
}

void launch_pose_solve(const Launch& L, int fp64, int iter) {
    if (fp64)
        hipLaunchKernelGGL(k_pose_solve<double>, dim3(L.grid[KK_ONE]), dim3(256), 0, L.s, L.B, iter);
    else
        hipLaunchKernelGGL(k_pose_solve<float>, dim3(L.grid[KK_ONE]), dim3(256), 0, L.s, L.B, iter);
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
__global__ void __launch_bounds__(256) k_shape(Batch B, int vo_sel, int vn_sel, int pn) {
    __shared__ float sdq[8 * (kMaxLinks + 1)];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_VERT, blockIdx.x, local)];
    const DevModel& m = S.m;
    const float4* __restrict__ v_old = S.verts[S.v_cur ^ vo_sel];
    const float4* __restrict__ v_new = S.verts[S.v_cur ^ vn_sel];
    const Vec3Buf n = S.normals;
    const Accum& a = S.a;
    const int src = phi_index(S, pn);
    const Vec3Buf phi = S.phi[src];
    const Vec3Buf phi_prev = S.phi[S.phi_prev];
    const Vec3Buf phi_out = S.phi[phi_next(src, S.phi_prev)];
    const float lphi = S.lphi, lnbr = S.lnbr, lt = S.lt, lw = S.lw;
    for (int q = threadIdx.x; q < 8 * m.L; q += blockDim.x) sdq[q] = S.dq[q];
    __syncthreads();
    int i = local * blockDim.x + threadIdx.x;
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
        const float4 vo = v_old[i], vn = v_new[i];
        T dx = (T)a.sx[i] * inv + ((T)vo.x - (T)vn.x);
        T dy = (T)a.sy[i] * inv + ((T)vo.y - (T)vn.y);
        T dz = (T)a.sz[i] * inv + ((T)vo.z - (T)vn.z);
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

void launch_shape(const Launch& L, int fp64, int v_old, int v_new, int pn) {
    const dim3 g(L.grid[KK_VERT]);
    if (fp64)
        hipLaunchKernelGGL(k_shape<double>, g, dim3(256), 0, L.s, L.B, v_old, v_new, pn);
    else
        hipLaunchKernelGGL(k_shape<float>, g, dim3(256), 0, L.s, L.B, v_old, v_new, pn);
}

}  // namespace trk
