// Forward kinematics of one pose in one workgroup (Section 3.1), shared by
// the FK kernel and the pose-step kernel.
#pragma once
#include "common.h"
#include "dq.h"

namespace trk {

// ---------------------------------------------------------------------------
// Forward kinematics (Section 3.1) in float64, one workgroup.
//
// Each joint first forms its local transform O_j H_j(theta_j) (Eq. 1 or 2);
// the chain products H_{0,j} = H_{0,P(j)} O_j H_j are then formed by pointer
// jumping: every joint repeatedly left-multiplies by the product held at its
// current ancestor and jumps to that ancestor's ancestor, so a tree of depth
// D needs ceil(log2 D) rounds (jt->rounds) instead of D dependent steps.
//
// Outputs (float32): the link offsets H_{l,Delta} = H_{0,l} (H^0_{0,l})^{-1}
// (8 per link) and, per joint k, the world-frame generator
//   Xi_k = H_{0,k} (dH_k/dtheta H_k^{-1}) H_{0,k}^{-1},
// i.e. H_{0,k} (z/2) H_{0,k}^* for a hinge and H_{0,k} (eps z/2) H_{0,k}^* for
// a prismatic, stored as its 6 vector components (real xyz, dual xyz) + pad.
// dH_{l,Delta}/dtheta_k = Xi_k H_{l,Delta} for every joint k on the chain of
// link l (the derivative blocks of Section 4.2).
// ---------------------------------------------------------------------------
// LDS workspace of fk_block (callers provide it, so that a kernel can
// overlay it on memory it no longer needs)
struct FkScratch {
    double M[2][kMaxJoints + 1][8];
    int A[2][kMaxJoints + 1];
};

__device__ __forceinline__ void fk_block(const JointTable* __restrict__ jt, int P, int L,
                                         const double* __restrict__ theta, float* __restrict__ dq,
                                         float* __restrict__ xi, FkScratch& ws) {
    double (*M)[kMaxJoints + 1][8] = ws.M;
    int (*A)[kMaxJoints + 1] = ws.A;
    const int t = threadIdx.x;
    for (int j = t; j < P; j += blockDim.x) {
        double th = theta[j];
        double Hj[8] = {1, 0, 0, 0, 0, 0, 0, 0};
        const double* z = jt->axis[j];
        if (jt->type[j] == 0) {
            double s, c;
            sincos(0.5 * th, &s, &c);
            Hj[0] = c; Hj[1] = s * z[0]; Hj[2] = s * z[1]; Hj[3] = s * z[2];
        } else {
            Hj[5] = 0.5 * th * z[0]; Hj[6] = 0.5 * th * z[1]; Hj[7] = 0.5 * th * z[2];
        }
        double loc[8];
        dqmul(jt->off[j], Hj, loc);
        for (int c = 0; c < 8; ++c) M[0][j][c] = loc[c];
        A[0][j] = jt->parent[j];
    }
    __syncthreads();
    int cur = 0;
    for (int round = 0; round < jt->rounds; ++round) {
        int nxt = cur ^ 1;
        for (int j = t; j < P; j += blockDim.x) {
            int a = A[cur][j];
            if (a >= 0) {
                double o[8];
                dqmul(M[cur][a], M[cur][j], o);
                for (int c = 0; c < 8; ++c) M[nxt][j][c] = o[c];
                A[nxt][j] = A[cur][a];
            } else {
                for (int c = 0; c < 8; ++c) M[nxt][j][c] = M[cur][j][c];
                A[nxt][j] = -1;
            }
        }
        __syncthreads();
        cur = nxt;
    }
    for (int j = t; j < P; j += blockDim.x) {
        const double* H = M[cur][j];
        double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const double* z = jt->axis[j];
        if (jt->type[j] == 0) { g[1] = 0.5 * z[0]; g[2] = 0.5 * z[1]; g[3] = 0.5 * z[2]; }
        else { g[5] = 0.5 * z[0]; g[6] = 0.5 * z[1]; g[7] = 0.5 * z[2]; }
        double hc[8], tmp[8], o[8];
        dqconj(H, hc);
        dqmul(H, g, tmp);
        dqmul(tmp, hc, o);
        float* dst = xi + 8 * j;
        dst[0] = (float)o[1]; dst[1] = (float)o[2]; dst[2] = (float)o[3];
        dst[3] = (float)o[5]; dst[4] = (float)o[6]; dst[5] = (float)o[7];
        dst[6] = 0.0f; dst[7] = 0.0f;
    }
    for (int l = t; l < L; l += blockDim.x) {
        double o[8];
        dqmul(M[cur][jt->link_joint[l]], jt->binv[l], o);
        for (int c = 0; c < 8; ++c) dq[8 * l + c] = (float)o[c];
    }
}

// The same forward kinematics with the constants read ahead of time (a
// kernel issues fk_prefetch early, so the reads overlap other work) and the
// pose taken from LDS.  Joint j's data sit in thread j, link l's in thread
// kLinkThread + l (so the joint and link outputs are formed side by side when
// the workgroup has kLinkThread + L threads).
constexpr int kLinkThread = 256;

struct FkJoint { double off[8], z[3]; int type, parent; };
struct FkLink { double binv[8]; int joint; };

__device__ __forceinline__ void fk_prefetch(const JointTable* __restrict__ jt, int P, int L, FkJoint& fj, FkLink& fl) {
    // every thread reads (at clamped indices; the others' values go unused),
    // so that no read waits under a branch, and as global reads, so that the
    // LDS work in between does not wait for them
    const int t = threadIdx.x;
    const int tj = min(t, P - 1), tl = min(max(t - kLinkThread, 0), L - 1);
#pragma unroll
    for (int c = 0; c < 8; ++c) fj.off[c] = ldg(&jt->off[tj][c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) fj.z[c] = ldg(&jt->axis[tj][c]);
    fj.type = ldg(&jt->type[tj]);
    fj.parent = ldg(&jt->parent[tj]);
#pragma unroll
    for (int c = 0; c < 8; ++c) fl.binv[c] = ldg(&jt->binv[tl][c]);
    fl.joint = ldg(&jt->link_joint[tl]);
}

__device__ __forceinline__ void fk_block_pre(int P, int L, int rounds, const double* __restrict__ sth,
                                             const FkJoint& fj, const FkLink& fl, float* __restrict__ dq,
                                             float* __restrict__ xi, FkScratch& ws) {
    double (*M)[kMaxJoints + 1][8] = ws.M;
    int (*A)[kMaxJoints + 1] = ws.A;
    const int t = threadIdx.x;
    if (t < P) {
        const double th = sth[t];
        double Hj[8] = {1, 0, 0, 0, 0, 0, 0, 0};
        if (fj.type == 0) {
            double s, c;
            sincos(0.5 * th, &s, &c);
            Hj[0] = c; Hj[1] = s * fj.z[0]; Hj[2] = s * fj.z[1]; Hj[3] = s * fj.z[2];
        } else {
            Hj[5] = 0.5 * th * fj.z[0]; Hj[6] = 0.5 * th * fj.z[1]; Hj[7] = 0.5 * th * fj.z[2];
        }
        double loc[8];
        dqmul(fj.off, Hj, loc);
        for (int c = 0; c < 8; ++c) M[0][t][c] = loc[c];
        A[0][t] = fj.parent;
    }
    __syncthreads();
    int cur = 0;
    for (int round = 0; round < rounds; ++round) {
        const int nxt = cur ^ 1;
        if (t < P) {
            const int a = A[cur][t];
            if (a >= 0) {
                double o[8];
                dqmul(M[cur][a], M[cur][t], o);
                for (int c = 0; c < 8; ++c) M[nxt][t][c] = o[c];
                A[nxt][t] = A[cur][a];
            } else {
                for (int c = 0; c < 8; ++c) M[nxt][t][c] = M[cur][t][c];
                A[nxt][t] = -1;
            }
        }
        __syncthreads();
        cur = nxt;
    }
    if (t < P) {
        const double* H = M[cur][t];
        double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (fj.type == 0) { g[1] = 0.5 * fj.z[0]; g[2] = 0.5 * fj.z[1]; g[3] = 0.5 * fj.z[2]; }
        else { g[5] = 0.5 * fj.z[0]; g[6] = 0.5 * fj.z[1]; g[7] = 0.5 * fj.z[2]; }
        double hc[8], tmp[8], o[8];
        dqconj(H, hc);
        dqmul(H, g, tmp);
        dqmul(tmp, hc, o);
        float* dst = xi + 8 * t;
        dst[0] = (float)o[1]; dst[1] = (float)o[2]; dst[2] = (float)o[3];
        dst[3] = (float)o[5]; dst[4] = (float)o[6]; dst[5] = (float)o[7];
        dst[6] = 0.0f; dst[7] = 0.0f;
    }
    const int l = t - kLinkThread;
    if (l >= 0 && l < L) {
        double o[8];
        dqmul(M[cur][fl.joint], fl.binv, o);
        for (int c = 0; c < 8; ++c) dq[8 * l + c] = (float)o[c];
    }
}

}  // namespace trk
