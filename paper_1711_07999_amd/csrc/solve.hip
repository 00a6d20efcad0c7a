// Pose step (Section 4.2) and per-vertex offset step (Section 4.3).
#include "common.h"
#include "dq.h"
#include "fk.h"
#include "surface.h"

namespace trk {

// ---------------------------------------------------------------------------
// Damped least squares (Marquardt): (A + lambda_k diag(A)) x = b with
// A = J^T J + (lambda_s S)^2 and b = J^T r + (lambda_s S)^2 Theta, solved by
// Cholesky; Theta <- Theta - x.  Parameters with A_kk == 0 (no observed vertex
// moves them) or marked inactive are frozen (x_k = 0).  A failed
// factorisation leaves Theta unchanged and flags the frame.
//
// One workgroup per stream.  The damped matrix (padded with identity rows to
// a multiple of 16) sits in LDS with b appended as an extra row, and is
// factored left-looking in 16-column panels: all four waves first subtract
// the contribution of the finished panels from the new one (dot products out
// of LDS), then wave 0 factors the panel in registers -- one row per lane,
// columns broadcast between lanes with readlane, so the column-to-column
// chain has no barrier.  The appended row becomes y = L^-1 b on the way
// (forward substitution for free).  Back substitution runs panel by panel in
// wave 0; the same workgroup then runs forward kinematics at the new pose.
// ---------------------------------------------------------------------------
constexpr int kPanel = 16;
constexpr int kNMax = kMaxJoints + 1;   // 128

// Dynamic LDS of the solve for padded size n (row stride n + 4, so rows are
// 16-byte aligned for vector access): the matrix with the right-hand-side
// row (reused for forward kinematics afterwards), x, 1 / L_jj, the frozen
// flags and the failure flag.
template <class T>
__host__ __device__ inline size_t solve_lds_bytes(int n) {
    size_t mat = sizeof(T) * (size_t)(n + 1) * (n + 4);
    if (mat < sizeof(FkScratch)) mat = sizeof(FkScratch);
    mat = (mat + 15) & ~size_t(15);
    return mat + 2 * sizeof(T) * n + sizeof(int) * (n + 1);
}

// 1/sqrt(d): the hardware estimate for float (1 ulp), IEEE for double
__device__ __forceinline__ float rsqrt_of(float d) { return __builtin_amdgcn_rsqf(d); }
__device__ __forceinline__ double rsqrt_of(double d) { return 1.0 / sqrt(d); }

// four consecutive elements from 16-byte aligned LDS
__device__ __forceinline__ void load4(const float* p, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double* o) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_bcast(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void store4(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}

constexpr size_t kSmallLds = 64 * 1024;

// BIG: an instance allowed more than 64 KB of LDS (P > 112 in float64); a
// kernel allowed that much is launched more slowly, so sizes below use the
// other instance
template <class T, bool BIG>
__global__ void __launch_bounds__(256) k_pose_solve(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int iter, int nmax) {
    const Batch B{bs, bp, bn};
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int ld = nmax + 4;   // row stride shared by the batch
    size_t mat = sizeof(T) * (size_t)(nmax + 1) * ld;
    if (mat < sizeof(FkScratch)) mat = sizeof(FkScratch);
    mat = (mat + 15) & ~size_t(15);
    T* M = reinterpret_cast<T*>(smem);
    FkScratch& fk_ws = *reinterpret_cast<FkScratch*>(smem);
    T* sx = reinterpret_cast<T*>(smem + mat);
    T* sdinv = sx + nmax;
    int* sfrozen = reinterpret_cast<int*>(sdinv + nmax);
    int& sfail = sfrozen[nmax];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_ONE, blockIdx.x, local)];
    const JointTable* __restrict__ jt = S.jt;
    const int PP = S.PP;
    const double* __restrict__ gram = S.gram;
    const float lambda_k = S.lambda_k;
    double* __restrict__ theta = S.theta;
    DevStats* st = S.st;
    const int P = S.m.P;   // (the table's copy: no dependent load through jt)
    const int n = (P + kPanel - 1) / kPanel * kPanel;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    // Every global read of the set-up is issued before any is used: the
    // strictly lower triangle (a quarter-wave per row, four rows at a time)
    // and, per parameter, its diagonal, right-hand side, prior and flags.
    const int q = tid & 15, row0 = tid >> 4;
    constexpr int kRows = 4;
    T raw[2][kRows][kNMax / 16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int a = 0; a < kRows; ++a) {
            const int r = row0 + 16 * (kRows * h + a);
#pragma unroll
            for (int u = 0; u < kNMax / 16; ++u) {
                const int c = q + 16 * u;
                raw[h][a][u] = (r < P && c < r) ? T(gram[r * PP + c]) : T(0);
            }
        }
    double gkk = 0.0, gkb = 0.0, prk = 0.0, thk = 0.0;
    int actk = 0;
    if (tid < P) {
        gkk = gram[tid * PP + tid];
        gkb = gram[tid * PP + P];
        prk = jt->prior[tid];
        thk = theta[tid];
        actk = jt->active[tid];
    }
    if (tid == 0) sfail = 0;
    if (tid < n) {
        const int fz = tid >= P || (gkk + prk == 0.0) || !actk;
        sfrozen[tid] = fz;
        M[n * ld + tid] = fz ? T(0) : T(gkb + prk * thk);
        M[tid * ld + tid] = fz ? T(1) : T((gkk + prk) * (1.0 + (double)lambda_k));
    }
    __syncthreads();
    // the damped, frozen and padded matrix (lower triangle)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int a = 0; a < kRows; ++a) {
            const int r = row0 + 16 * (kRows * h + a);
            if (r >= n) continue;
            const bool fr = sfrozen[r] != 0;
#pragma unroll
            for (int u = 0; u < kNMax / 16; ++u) {
                const int c = q + 16 * u;
                if (c < r) M[r * ld + c] = (fr || sfrozen[c]) ? T(0) : raw[h][a][u];
            }
        }
    __syncthreads();

    for (int c0 = 0; c0 < n; c0 += kPanel) {
        // (1) A[r][c] -= sum_{k < c0} L[r][k] L[c][k] for the panel's columns,
        //     rows c0..n (row n: b -> y)
        if (c0 > 0) {
            const int rows = n + 1 - c0;
            for (int e = tid; e < rows * kPanel; e += 256) {
                const int r = c0 + e / kPanel, c = c0 + (e & (kPanel - 1));
                if (c > r) continue;
                const T* Lr = M + r * ld;
                const T* Lc = M + c * ld;
                T acc[4] = {T(0), T(0), T(0), T(0)};
                for (int k = 0; k < c0; k += 4) {
                    T xr[4], xc[4];
                    load4(Lr + k, xr);
                    load4(Lc + k, xc);
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[t] += xr[t] * xc[t];
                }
                M[r * ld + c] -= (acc[0] + acc[1]) + (acc[2] + acc[3]);
            }
            __syncthreads();
        }
        // (2) factor the panel in wave 0: lane l holds rows c0 + l and
        //     c0 + 64 + l; every lane carries the right-hand-side row
        if (wid == 0) {
            const int r0 = c0 + lane, r1 = c0 + 64 + lane;
            const bool h0 = r0 < n, h1 = r1 < n;
            T a0[kPanel], a1[kPanel], ab[kPanel];
#pragma unroll
            for (int j = 0; j < kPanel; j += 4) {
                if (h0) load4(M + r0 * ld + c0 + j, a0 + j);
                else a0[j] = a0[j + 1] = a0[j + 2] = a0[j + 3] = T(0);
                if (h1) load4(M + r1 * ld + c0 + j, a1 + j);
                else a1[j] = a1[j + 1] = a1[j + 2] = a1[j + 3] = T(0);
                load4(M + n * ld + c0 + j, ab + j);
            }
            const bool two = c0 + 64 < n;   // the second row set holds rows
            bool ok = true;
#pragma unroll
            for (int j = 0; j < kPanel; ++j) {
                const T d = lane_bcast(a0[j], j);
                ok = ok && (d > T(0));
                const T inv = ok ? rsqrt_of(d) : T(1);
                // column j of L: the diagonal, then the rows below it; y_j.
                // Lanes at or above the diagonal keep their (unused) entries.
                const T lj = lane > j ? a0[j] * inv : T(0);
                a0[j] = lane == j ? d * inv : (lane > j ? lj : a0[j]);
                a1[j] *= inv;
                ab[j] *= inv;
                if (lane == 0) sdinv[c0 + j] = inv;
                if (two) {
#pragma unroll
                    for (int c = j + 1; c < kPanel; ++c) {
                        const T lcj = lane_bcast(lj, c);
                        a0[c] -= lj * lcj;
                        a1[c] -= a1[j] * lcj;
                        ab[c] -= ab[j] * lcj;
                    }
                } else {
#pragma unroll
                    for (int c = j + 1; c < kPanel; ++c) {
                        const T lcj = lane_bcast(lj, c);
                        a0[c] -= lj * lcj;
                        ab[c] -= ab[j] * lcj;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kPanel; ++j) {
                if (h0 && r0 >= c0 + j) M[r0 * ld + c0 + j] = a0[j];
                if (h1) M[r1 * ld + c0 + j] = a1[j];
                if (lane == 0) M[n * ld + c0 + j] = ab[j];
            }
            if (!ok && lane == 0) sfail = 1;
        }
        __syncthreads();
        if (sfail) break;
    }
    const bool fail = sfail != 0;
    if (!fail && wid == 0) {
        // back substitution L^T x = y, panel by panel from the last
        for (int c0 = n - kPanel; c0 >= 0; c0 -= kPanel) {
            // t_c = y_c - sum_{r >= c0 + 16} L[r][c] x_r for the panel's 16 columns:
            // lanes 16 g + l take rows r = c0 + 16 + g, +4, ...
            const int l = lane & (kPanel - 1), g = lane >> 4;
            T t = T(0);
            for (int r = c0 + kPanel + g; r < n; r += 4) t += M[r * ld + c0 + l] * sx[r];
            t += __shfl_xor(t, 16);
            t += __shfl_xor(t, 32);
            t = M[n * ld + c0 + l] - t;
            // upper-triangular 16x16 solve with L_pp^T in registers (column l)
            T lc[kPanel];
#pragma unroll
            for (int j = 0; j < kPanel; ++j) lc[j] = j >= l ? M[(c0 + j) * ld + c0 + l] : T(0);
#pragma unroll
            for (int j = kPanel - 1; j >= 0; --j) {
                const T xj = lane_bcast(t, j) * sdinv[c0 + j];
                t = l < j ? t - lc[j] * xj : (l == j ? xj : t);
            }
            if (lane < kPanel) sx[c0 + lane] = t;
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    if (!fail) {
        if (wid == 0) {
            double part = 0.0;
            for (int k = lane; k < P; k += 64) {
                const double x = sfrozen[k] ? 0.0 : (double)sx[k];
                S.step[k] = x;
                theta[k] -= x;
                part += x * x;
            }
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
            if (lane == 0) {
                st->step_norm[S.iter + iter] = (float)sqrt(part);
                st->energy[S.iter + iter] = (float)gram[P * PP + P];
            }
        }
    } else if (tid == 0) {
        st->status = -4;
        st->energy[S.iter + iter] = (float)gram[P * PP + P];
        st->step_norm[S.iter + iter] = 0.0f;
    }
    __syncthreads();
    fk_block(jt, P, S.m.L, theta, S.dq, S.xi, fk_ws);
}

// ---------------------------------------------------------------------------
// Tree form of the same solve.  J_ik vanishes unless joint k lies on the
// chain of a link weighting vertex i (Section 4.2), so A_kj vanishes unless
// some vertex's chains hold both joints: limbs do not touch each other, only
// their common ancestors.  Eliminated children first, the factor stays
// inside that pattern and its elimination tree follows the skeleton (the
// host plan, TreePlan).  Each supernode -- a chain of the elimination tree --
// owns a dense front: its pivot rows, the later rows they touch, and the
// right-hand side as one more row.  Level by level, each wave takes its
// supernodes: it adds the children's update blocks to the front, loads one
// front row per lane into registers, factors the pivots with lane
// broadcasts (the right-hand-side row turns into y on the way, the rest of
// the front into the update block for the parent) and stores the front
// back; 1 / L_jj goes into the front's spare last column.  Back
// substitution walks the levels downwards.  Only structural zeros are
// skipped: the arithmetic per entry is that of the dense form.
// ---------------------------------------------------------------------------
// Dynamic LDS of the tree form: the fronts (reused for forward kinematics),
// a copy of the plan, x, the damped diagonal, the right-hand side, flags.
template <class T>
__host__ __device__ inline size_t tree_front_bytes(int elems) {
    size_t mat = sizeof(T) * (size_t)elems;
    if (mat < sizeof(FkScratch)) mat = sizeof(FkScratch);
    return (mat + 15) & ~size_t(15);
}
template <class T>
__host__ __device__ inline size_t tree_lds_bytes(int elems, int words) {
    return tree_front_bytes<T>(elems) + 16 * (size_t)((words + 3) / 4) + sizeof(T) * kNMax +
           sizeof(double) * (kNMax + kSolveWaves) + sizeof(T) * 64 * kSolveWaves + 16;
}

bool tree_solve_fits(int elems, int words) { return tree_lds_bytes<double>(elems, words) <= kSmallLds; }

// Factor the np pivots of a front of f rows (+ the right-hand-side row f),
// row-major with FW columns, FW > f.  Lane i holds row i in registers; each
// pivot's update also shifts the row one column to the left, so the pivot
// column is always r[0].  The new column of L goes to the wave's buffer
// `wb`, written shifted so that every lane reads the multipliers of the
// columns still to come from its start (wide broadcast reads, one lane
// broadcast per pivot).  Column j of L is stored as it is found, the update
// block (columns np..f-1 of rows np..f) at the end, and 1 / L_jj into the
// spare column FW - 1.
template <class T, int FW>
__device__ __forceinline__ void tree_factor(T* Fr, T* wb, int np, int f, int lane, bool& ok) {
    T r[FW];
    const bool live = lane <= f;
#pragma unroll
    for (int c = 0; c < FW; c += 4) {
        if (live) load4(Fr + lane * FW + c, r + c);
        else r[c] = r[c + 1] = r[c + 2] = r[c + 3] = T(0);
    }
    T myinv = T(0);
    for (int j = 0; j < np; ++j) {
        const T d = lane_bcast(r[0], j);
        ok = ok && (d > T(0));
        const T inv = ok ? rsqrt_of(d) : T(1);
        // column j of L below the diagonal (the right-hand-side row: y_j)
        const T lj = lane > j ? r[0] * inv : T(0);
        if (lane == j) myinv = inv;
        // masked lanes store to wb[63], which no lane reads
        *(live && lane >= j ? Fr + lane * FW + j : wb + 63) = lane == j ? d * inv : lj;
        *(lane > j ? wb + (lane - j - 1) : wb + 63) = lj;   // wb[k] = L_{j+1+k, j}; lanes j+1..63 cover k < FW
        T cv[FW];
#pragma unroll
        for (int c = 0; c < FW; c += 4) load4(wb + c, cv + c);
#pragma unroll
        for (int c = 1; c < FW; ++c) r[c - 1] = r[c] - lj * cv[c - 1];
        r[FW - 1] = T(0);
    }
    const int nU = f - np;
#pragma unroll
    for (int c = 0; c < FW - 1; ++c)
        if (c < nU && live) Fr[lane * FW + np + c] = r[c];
    if (lane < np) Fr[lane * FW + FW - 1] = myinv;
}

// L^T x = y for the front's pivots (row stride fw), given x of its later
// rows; lane c < np takes pivot c.  `row` maps front rows to joints; `wb`
// is the wave's buffer.
template <class T>
__device__ __forceinline__ void tree_back(const T* Fr, T* wb, int np, int f, int fw, const unsigned char* row,
                                          T* sx, int lane) {
    const int nU = f - np;
    // x of the later rows, broadcast through the wave's buffer
    if (lane < nU) wb[lane] = sx[row[np + lane]];
    const int cl = lane < np ? lane : 0;
    T t = Fr[f * fw + cl];
    // four independent partial sums, so four rows' loads are in flight
    T t1 = T(0), t2 = T(0), t3 = T(0);
    int k = 0;
    for (; k + 4 <= nU; k += 4) {
        const T* R = Fr + (np + k) * fw + cl;
        t -= R[0] * wb[k];
        t1 -= R[fw] * wb[k + 1];
        t2 -= R[2 * fw] * wb[k + 2];
        t3 -= R[3 * fw] * wb[k + 3];
    }
    for (; k < nU; ++k) t -= Fr[(np + k) * fw + cl] * wb[k];
    t = (t + t1) + (t2 + t3);
    // the pivots' own triangle, last pivot first
    for (int j = np - 1; j >= 0; --j) {
        const T dinv = Fr[j * fw + fw - 1];
        const T lij = Fr[j * fw + cl];
        const T xj = lane_bcast(t, j) * dinv;
        t = lane < j ? t - lij * xj : (lane == j ? xj : t);
    }
    if (lane < np) sx[row[lane]] = t;
}

template <class T>
__global__ void __launch_bounds__(kSolveThreads) k_pose_solve_tree(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int iter, int elems_max, int words_max) {
    const Batch B{bs, bp, bn};
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const size_t mat = tree_front_bytes<T>(elems_max);
    T* Fs = reinterpret_cast<T*>(smem);
    FkScratch& fk_ws = *reinterpret_cast<FkScratch*>(smem);
    uint32_t* lb = reinterpret_cast<uint32_t*>(smem + mat);   // the plan's blob, copied to LDS
    T* sx = reinterpret_cast<T*>(smem + mat + 16 * (size_t)((words_max + 3) / 4));
    double* sth = reinterpret_cast<double*>(sx + kNMax);      // the new pose
    double* spart = sth + kNMax;                               // per-wave sums of x^2
    T* wbase = reinterpret_cast<T*>(spart + kSolveWaves);
    int& sfail = *reinterpret_cast<int*>(wbase + 64 * kSolveWaves);
    int local;
    const Slot& S = B.slots[slot_of(B, KK_ONE, blockIdx.x, local)];
    const TreeRef& tr = S.tree;
    const JointTable* __restrict__ jt = S.jt;
    const int PP = S.PP;
    const double* __restrict__ gram = S.gram;
    double* __restrict__ theta = S.theta;
    DevStats* st = S.st;
    const int P = S.m.P, NL = S.m.L;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    T* wb = wbase + 64 * wid;   // this wave's broadcast buffer

    // set-up: every global read is issued before any is used -- the fronts'
    // starting image (from the Gram reduction), the plan, and per joint the
    // pose and whether it is frozen
    const int elems = tr.elems;   // even: rows are multiples of 8 wide
    const double2* __restrict__ img = reinterpret_cast<const double2*>(tr.fimg);
    // (unconditional loads at clamped indices, the unused ones dropped after:
    // a load under a condition is waited for inside it, one after another)
    constexpr int kPre = 8;
    double2 iv[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) iv[k] = img[min(tid + kSolveThreads * k, elems / 2 - 1)];
    const uint4* __restrict__ bsrc = reinterpret_cast<const uint4*>(tr.blob);
    const int nw4 = (tr.nwords + 3) / 4;
    const uint4 bw = bsrc[min(tid, nw4 - 1)];
    const int tp = min(tid, P - 1);
    const double th0 = theta[tp], gdiag = gram[tp * PP + tp], prior = jt->prior[tp];
    const int act = jt->active[tp];
    const double energy = gram[P * PP + P];
    const int rounds = jt->rounds;
    const double thk = tid < P ? th0 : 0.0;
    const int fz = tid < P ? (int)((gdiag + prior == 0.0) | !act) : 1;
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        const int e = tid + kSolveThreads * k;
        if (2 * e < elems) {
            Fs[2 * e] = T(iv[k].x);
            Fs[2 * e + 1] = T(iv[k].y);
        }
    }
    for (int e = tid + kSolveThreads * kPre; 2 * e < elems; e += kSolveThreads) {
        const double2 v = img[e];
        Fs[2 * e] = T(v.x);
        Fs[2 * e + 1] = T(v.y);
    }
    if (tid < nw4) reinterpret_cast<uint4*>(lb)[tid] = bw;
    for (int i = tid + kSolveThreads; i < nw4; i += kSolveThreads) reinterpret_cast<uint4*>(lb)[i] = bsrc[i];
    if (tid == 0) sfail = 0;
    __syncthreads();

    // factor, level by level
    const int nlev = tr.nlev;
    const int* wstart = reinterpret_cast<const int*>(lb);
    const int* sched = wstart + tr.o_sched;
    const FrontRec* fronts = reinterpret_cast<const FrontRec*>(lb + tr.o_front);
    const unsigned char* lbytes = reinterpret_cast<const unsigned char*>(lb);
    bool ok = true;
    for (int l = 0; l < nlev; ++l) {
        const int q1 = wstart[l * kSolveWaves + wid + 1];
        for (int q = wstart[l * kSolveWaves + wid]; q < q1; ++q) {
            const FrontRec F = fronts[sched[q]];
            T* Fr = Fs + F.off;
            // the children's update blocks, 64 entries a round (each parent
            // entry at most once per round, children in a fixed order)
            for (int r = 0; r < F.nround; ++r) {
                const uint32_t a = lb[F.amap0 + 64 * r + lane];
                const uint32_t src = a & 0xFFFFu, dst = a >> 16;
                if (dst != 0xFFFFu) Fs[dst] += Fs[src];
            }
            switch (F.fw) {
                case 8: tree_factor<T, 8>(Fr, wb, F.np, F.f, lane, ok); break;
                case 16: tree_factor<T, 16>(Fr, wb, F.np, F.f, lane, ok); break;
                case 24: tree_factor<T, 24>(Fr, wb, F.np, F.f, lane, ok); break;
                default: tree_factor<T, 32>(Fr, wb, F.np, F.f, lane, ok); break;
            }
        }
        if (!ok && lane == 0) sfail = 1;
        __syncthreads();
    }
    const bool fail = sfail != 0;
    // forward kinematics' constants, read while the back substitution runs
    FkJoint fj;
    FkLink fl;
    fk_prefetch(jt, P, NL, fj, fl);
    if (!fail) {
        for (int l = nlev - 1; l >= 0; --l) {
            const int q1 = wstart[l * kSolveWaves + wid + 1];
            for (int q = wstart[l * kSolveWaves + wid]; q < q1; ++q) {
                const FrontRec F = fronts[sched[q]];
                tree_back<T>(Fs + F.off, wb, F.np, F.f, F.fw, lbytes + F.row0, sx, lane);
            }
            __syncthreads();
        }
    }
    // the step: Theta <- Theta - x (frozen parameters keep their value)
    const double x = (tid < P && !fail && !fz) ? (double)sx[tid] : 0.0;
    if (tid < P) {
        const double th = thk - x;
        sth[tid] = th;
        if (!fail) {
            stg(S.step + tid, x);
            stg(theta + tid, th);
        }
    }
    double part = x * x;
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) spart[wid] = part;
    __syncthreads();
    if (tid == 0) {
        double norm2 = 0.0;
        for (int w = 0; w < kSolveWaves; ++w) norm2 += spart[w];
        st->energy[S.iter + iter] = (float)energy;
        st->step_norm[S.iter + iter] = fail ? 0.0f : (float)sqrt(norm2);
        if (fail) st->status = -4;
    }
    fk_block_pre(P, NL, rounds, sth, fj, fl, S.dq, S.xi, fk_ws);
}

// let the BIG instances take the largest system (P = 127, float64: about
// 136 KB of LDS)
bool prepare_pose_solve() {
    bool ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_pose_solve<double, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)solve_lds_bytes<double>(kNMax)) == hipSuccess;
    ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_pose_solve<float, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)solve_lds_bytes<float>(kNMax)) == hipSuccess && ok;
    return ok;
}

template <class T>
void launch_pose_solve_t(const Launch& L, int iter) {
    if (L.solve_elems > 0) {
        const size_t bytes = tree_lds_bytes<T>(L.solve_elems, L.solve_words);
        launch_kernel(L, true, true, k_pose_solve_tree<T>, dim3(L.grid[KK_ONE]), dim3(kSolveThreads), bytes, L.B.slots, L.B.pre, L.B.n,
                      iter, L.solve_elems, L.solve_words);
        return;
    }
    const int n = L.solve_n;
    const size_t bytes = solve_lds_bytes<T>(n);
    if (bytes <= kSmallLds)
        launch_kernel(L, true, true, k_pose_solve<T, false>, dim3(L.grid[KK_ONE]), dim3(256), bytes, L.B.slots, L.B.pre, L.B.n, iter, n);
    else
        launch_kernel(L, true, true, k_pose_solve<T, true>, dim3(L.grid[KK_ONE]), dim3(256), bytes, L.B.slots, L.B.pre, L.B.n, iter, n);
}

void launch_pose_solve(const Launch& L, int fp64, int iter) {
    if (fp64) launch_pose_solve_t<double>(L, iter);
    else launch_pose_solve_t<float>(L, iter);
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
__global__ void __launch_bounds__(256) k_shape(const Slot* __restrict__ bs, const int* __restrict__ bp, int bn, int vo_sel, int vn_sel, int pn, int next, int bsel) {
    const Batch B{bs, bp, bn};
    __shared__ float sdq[8 * (kMaxLinks + 1)];
    int local;
    const Slot& S = B.slots[slot_of(B, KK_VERT64, blockIdx.x, local)];
    const DevModel& m = S.m;
    const float4* __restrict__ v_old = S.verts[S.v_cur ^ vo_sel];
    const float4* __restrict__ v_new = S.verts[S.v_cur ^ vn_sel];
    const Accum& a = S.a;
    const int src = phi_index(S, pn);
    const Vec3Buf phi = S.phi[src];
    const Vec3Buf phi_prev = S.phi[S.phi_prev];
    const Vec3Buf phi_out = S.phi[phi_next(src, S.phi_prev)];
    const float lphi = S.lphi, lnbr = S.lnbr, lt = S.lt, lw = S.lw;
    const bool counted = selected(S, next);
    const CountRefs cr = count_refs(S, bsel);
    // the slot fields used after the first loads, read here (into scalar
    // registers) rather than each where it is used, behind its own wait
    const bool linear = wave_uniform(S.blend) == kBlendLinear;
    uint32_t* const acnt = wave_uniform(a.cnt);
    long long* const asx = wave_uniform(a.sx);
    long long* const asy = wave_uniform(a.sy);
    long long* const asz = wave_uniform(a.sz);
    float* const pox = wave_uniform(phi_out.x);
    float* const poy = wave_uniform(phi_out.y);
    float* const poz = wave_uniform(phi_out.z);
    float4* const vnext = wave_uniform(S.verts[S.v_cur ^ vn_sel ^ 1]);
    const int i = local * blockDim.x + threadIdx.x;
    const bool live = i < m.V;
    const int ii = live ? i : 0;   // lanes past the end read vertex 0 and store nothing
    // every per-vertex load that does not wait on another goes out first,
    // ahead of the link table's copy (global reads: the barrier does not wait
    // for them), so their latencies overlap the copy's and each other's
    const uint32_t c0 = ldg(a.cnt + ii);
    const float px0 = ldg(phi.x + ii), py0 = ldg(phi.y + ii), pz0 = ldg(phi.z + ii);
    const float qx0 = ldg(phi_prev.x + ii), qy0 = ldg(phi_prev.y + ii), qz0 = ldg(phi_prev.z + ii);
    const int4 nb = ldg(m.nbr + ii);
    const float4 vo = ldg_xyz(v_old + ii), vn = ldg_xyz(v_new + ii);
    const long long ax = ldg(a.sx + ii), ay = ldg(a.sy + ii), az = ldg(a.sz + ii);
    const float4 wv = ldg(m.w + ii);
    const uint32_t lk = ldg(m.links + ii);
    const float rx = ldg(m.rx + ii), ry = ldg(m.ry + ii), rz = ldg(m.rz + ii);
    FanIn fan;
    vertex_fan_load(m, v_new, i, live, fan);   // not waiting for the count
    copy_to_lds(sdq, S.dq, 8 * m.L);
    __syncthreads();
    vertex_fan_settle(fan, live);
    const uint32_t c = live ? c0 : 0u;
    const T px = px0, py = py0, pz = pz0;
    const T qx = qx0, qy = qy0, qz = qz0;
    const int nbs[4] = {nb.x, nb.y, nb.z, nb.w};
    T nphi[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = nbs[q] < 0 ? ii : nbs[q];
        nphi[q][0] = (T)ldg(phi.x + j); nphi[q][1] = (T)ldg(phi.y + j); nphi[q][2] = (T)ldg(phi.z + j);
    }
    float nx, ny, nz;
    vertex_normal_fan(m, v_new, i, live && c > 0u, fan, nx, ny, nz);   // the whole wave
    // lanes past the end go on with vertex 0's values (count 0) and store nothing
    T u[3] = {T(0), T(0), T(0)};
    T r = T(0);
    float H[8];
    if (!linear) dq_blend(sdq, wv, lk, H);
    if (c > 0u) {
        if ((nx * nx + ny * ny + nz * nz) > 0.0f) {
            // dr/dphi = -(dv/dx)^T n: the blend's rotation, or for the linear
            // blend the weighted sum of the links' rotations
            T R[9];
            if (!linear) {
                quat_matrix<T>(H, R);
            } else {
                const float ws[4] = {wv.x, wv.y, wv.z, wv.w};
                for (int q = 0; q < 9; ++q) R[q] = T(0);
                for (int k = 0; k < 4; ++k) {
                    const int l = (lk >> (8 * k)) & 0xFF;
                    if (l == 0xFF) continue;
                    T Rl[9];
                    quat_matrix<T>(sdq + 8 * l, Rl);
                    for (int q = 0; q < 9; ++q) R[q] += (T)ws[k] * Rl[q];
                }
            }
            for (int q = 0; q < 3; ++q) u[q] = -(R[q] * nx + R[3 + q] * ny + R[6 + q] * nz);
            const T inv = T(1) / ((T)c * T(4294967296.0));
            T dx = (T)ax * inv + ((T)vo.x - (T)vn.x);
            T dy = (T)ay * inv + ((T)vo.y - (T)vn.y);
            T dz = (T)az * inv + ((T)vo.z - (T)vn.z);
            r = (T)nx * dx + (T)ny * dy + (T)nz * dz;
        }
    }
    // this is the association's last reader: clear for the next one
    if (live) {
        stg(acnt + i, 0u);
        stg(asx + i, 0ll); stg(asy + i, 0ll); stg(asz + i, 0ll);
    }
    T alpha = (T)lphi + (T)lt;
    T g[3] = {u[0] * r + (T)lphi * px + (T)lt * (px - qx),
              u[1] * r + (T)lphi * py + (T)lt * (py - qy),
              u[2] * r + (T)lphi * pz + (T)lt * (pz - qz)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (nbs[q] < 0) continue;
        alpha += (T)lnbr;
        g[0] += (T)lnbr * (px - nphi[q][0]);
        g[1] += (T)lnbr * (py - nphi[q][1]);
        g[2] += (T)lnbr * (pz - nphi[q][2]);
    }
    T M[9];
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) M[3 * p + q] = u[p] * u[q] + (p == q ? alpha : T(0));
    for (int p = 0; p < 3; ++p) M[4 * p] *= (T(1) + (T)lw);
    T xs[3];
    solve3(M, g, xs);
    const float fx = (float)(px - xs[0]), fy = (float)(py - xs[1]), fz = (float)(pz - xs[2]);
    if (live) {
        stg(pox + i, fx);
        stg(poy + i, fy);
        stg(poz + i, fz);
    }
    if (counted) {
        // the next iteration's surface: skin the new offsets (same blend) into
        // the buffer not read here by other vertices, and count it
        float ox, oy, oz;
        if (linear) lbs_apply(sdq, wv, lk, rx + fx, ry + fy, rz + fz, ox, oy, oz);
        else dq_apply(H, rx + fx, ry + fy, rz + fz, ox, oy, oz);
        const float4 q = make_float4(ox, oy, oz, 0.0f);
        if (live) stg(vnext + i, q);
        count_vertex(cr, i, q, live, false);   // the whole wave
    }
}

void launch_shape(const Launch& L, int fp64, int v_old, int v_new, int pn, int next, int bsel) {
    // one wave per workgroup: the vertices spread over every compute unit
    const dim3 g(L.grid[KK_VERT64]);
    if (fp64)
        launch_kernel(L, true, true, k_shape<double>, g, dim3(64), 0, L.B.slots, L.B.pre, L.B.n, v_old, v_new, pn, next, bsel);
    else
        launch_kernel(L, true, true, k_shape<float>, g, dim3(64), 0, L.B.slots, L.B.pre, L.B.n, v_old, v_new, pn, next, bsel);
}

}  // namespace trk
