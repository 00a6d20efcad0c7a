// Internal declarations shared by the HIP translation units of libtrack.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace trk {

constexpr int kMaxJoints = 127;
constexpr int kMaxLinks = 255;
constexpr int kPPMax = 128;          // padded Gram size (P + 1 rounded up to 16)
constexpr float kZNear = 1e-3f;      // vertices at z <= kZNear are not candidates
constexpr double kFix = 4294967296.0;  // 2^32: fixed-point quantum of the offsets (m)
constexpr int kNeRows = 128;         // vertices per normal-equation chunk

// Joint and link tables (device copy, built once per model on the host).
struct JointTable {
    int P, L;
    int parent[kMaxJoints + 1];
    int type[kMaxJoints + 1];
    double axis[kMaxJoints + 1][3];
    double off[kMaxJoints + 1][8];     // fixed offset O_j as a dual quaternion
    int link_joint[kMaxLinks + 1];
    double binv[kMaxLinks + 1][8];     // (H^0_{0,link joint})^{-1}
    uint32_t anc[kMaxLinks + 1][4];    // joints on the chain of each link
    double prior[kMaxJoints + 1];      // (lambda_s S_k)^2
    int active[kMaxJoints + 1];
};

// Mesh, weights and tables in structure-of-arrays device form.
struct DevModel {
    int P, L, V, F;
    const float *rx, *ry, *rz;     // template vertices
    const float4 *w;               // weights, padded to four
    const uint32_t *links;         // four link bytes per vertex, 0xFF = unused
    const int4 *nbr;               // neighbours, -1 = none
    const uint32_t *fan_off;       // [V+1] incident-face list per vertex
    const int2 *fan;               // (b, c) with face (i, b, c) counter-clockwise
};

struct DevCam {
    int W, H, tiles_x, tiles_y;
    float fx, fy, cx, cy;
    float lb_c1;   // lower bound of the 3-D distance per pixel ring, per metre of depth
};

// Per-iteration bookkeeping written by the kernels and read back per frame.
struct DevStats {
    int n_valid_px, n_assoc_px, n_obs_verts, status;
    float energy[256];
    float step_norm[256];
};

// Offset and normal buffers: SoA x, y, z of V floats each (skinned vertices
// are float4 (x, y, z, 0) so that neighbour gathers are single loads).
struct Vec3Buf { float *x, *y, *z; };
struct CVec3Buf { const float *x, *y, *z; };
inline CVec3Buf cview(const Vec3Buf& b) { return {b.x, b.y, b.z}; }

// Fixed-point per-vertex accumulators of the association.
struct Accum {
    uint32_t* cnt;           // pixels per vertex
    long long *sx, *sy, *sz; // sum of (p - v) in units of 2^-32 m
};

// Bucket (index/z-buffer) storage; pixels are numbered tile-major: 8x8
// tiles in row-major order, 64 pixels per tile in Morton order.
struct Buckets {
    uint32_t* pcnt;    // [Npad] vertices per pixel
    uint32_t* pzmin;   // [Npad] float bits of the smallest vertex z
    uint32_t* pzmax;   // [Npad] float bits of the largest vertex z
    uint4* rec;        // [Npad] (offset, count, zmin bits, zmax bits)
    uint32_t* tsum;    // [tiles] vertices per tile
    uint32_t* toff;    // [tiles] exclusive prefix of tsum
    float2* tz;        // [tiles] z range of the tile
    int* vpix;         // [V] bucket of each vertex or -1
    uint32_t* vslot;   // [V] rank inside its bucket
    float4* sorted;    // [V] (x, y, z, vertex id bits) grouped by bucket
    uint4* cellrec;    // [tiles*4] per 4x4 cell: (offset, count, zmin bits, zmax bits)
    int4* bstat;       // [tiles] valid, matched, newly observed pixels per tile
};

// Association launch shape: one workgroup per 8x8 tile.
inline int assoc_blocks(int tiles_x, int tiles_y) { return tiles_x * tiles_y; }

// ---- launchers (each defined next to its kernels) -------------------------
void launch_fk(hipStream_t s, const JointTable* jt, const double* theta, float* dq, float* xi);
void launch_skin(hipStream_t s, const DevModel& m, const float* dq, CVec3Buf phi, float4* v);
void launch_normals(hipStream_t s, const DevModel& m, const float4* v, Vec3Buf n);
void launch_clear(hipStream_t s, int npad, const Buckets& b, int V, const Accum& a, DevStats* st);
void launch_bucket(hipStream_t s, const DevCam& c, int V, const float4* v, const Buckets& b);
void launch_associate(hipStream_t s, const DevCam& c, float tau, const float* depth, const float* xyz,
                      const Buckets& b, const Accum& a, const float4* verts, int32_t* assoc);
int ne_grid(int V);
void launch_normal_eq(hipStream_t s, const DevModel& m, int PP, int gram_mode, const float* dq,
                      const float* xi, const uint32_t* anc_dev, const float4* v, CVec3Buf n, CVec3Buf phi,
                      const Accum& a, float* partials, int grid);
void launch_gram_reduce(hipStream_t s, int PP, int nparts, const float* partials, double* gram);
void launch_pose_solve(hipStream_t s, const JointTable* jt, int PP, const double* gram, float lambda_k,
                       int fp64, double* theta, double* step, DevStats* st, int iter, float* dq, float* xi);
void launch_shape(hipStream_t s, const DevModel& m, const float* dq, const float4* v_old, const float4* v_new,
                  CVec3Buf n, const Accum& a, CVec3Buf phi, CVec3Buf phi_prev, Vec3Buf phi_out,
                  float lphi, float lnbr, float lt, float lw, int fp64);
void launch_copy3(hipStream_t s, int V, CVec3Buf src, Vec3Buf dst);
void launch_frame_begin(hipStream_t s, int P, const double* theta, double* theta_backup, DevStats* st);

}  // namespace trk
