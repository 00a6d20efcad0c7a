// Internal declarations shared by the HIP translation units of libtrack.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>
#include <algorithm>

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
    int rounds;                        // ceil(log2(longest joint chain))
};

// Tree-ordered factorisation of the pose system (built on the host from the
// skeleton and the skin weights, read by the pose-solve kernel).  Joints are
// eliminated children first; chains of the elimination tree form supernodes,
// each with a dense front: its pivot rows, the later rows they touch, and the
// right-hand side as a last row, stored row-major with `fw` columns.
constexpr int kFrontRows = 32;       // rows of a front, right-hand side included
constexpr int kSolveWaves = 8;       // waves of the tree-form pose-solve workgroup
constexpr int kSolveThreads = 64 * kSolveWaves;
constexpr int kFrontWords = 8;       // words of a front record in the blob

// A front record: storage offset, pivots, rows (without the right-hand
// side), row width, first assembly word and number of 64-entry assembly
// rounds, byte offset of its row-to-joint map in the blob.
struct FrontRec { int off, np, f, fw, amap0, nround, row0, pad; };

// What the kernels read of a stream's tree plan (in its slot, so that no
// read waits on another).
struct TreeRef {
    const uint32_t* blob;            // TreePlan::blob
    double* fimg;                    // [elems] the fronts as the solve starts them, written by the
                                     // Gram reduction (damped, frozen); zero outside the entries
    const int* gfmap;                // [PP*PP] Gram position (at or above the diagonal, or the
                                     // right-hand side) -> front storage index, -1 none; null: dense form
    int nwords, nlev, elems, o_sched, o_front;
};

struct alignas(16) TreePlan {
    int ok;                          // the tree form applies to this model
    int nsn, nlev, elems;            // supernodes, levels, front storage (elements)
    int nwords;                      // words of `blob`
    int o_sched, o_front;            // word offsets of the schedule and the front records
    // what the kernel copies to LDS: per level and wave the first schedule
    // entry (wstart, kSolveWaves * nlev + 1 words), the schedule, the front
    // records, the assembly rounds (per parent, 64 entries a round: child
    // storage index | parent storage index << 16, 0xFFFF = none; a parent
    // entry appears at most once per round, children's shares in child
    // order), then the row maps (bytes)
    const uint32_t* blob;
};

constexpr int kFanInline = 8;   // incident faces of a vertex held in the inline (per-slot) table

// Mesh, weights and tables in structure-of-arrays device form.
constexpr int kBlendLinear = 1;   // TRACK_BLEND_LINEAR

struct DevModel {
    int P, L, V, F;
    const float *rx, *ry, *rz;     // template vertices
    const float4 *w;               // weights, padded to four
    const uint32_t *links;         // four link bytes per vertex, 0xFF = unused
    const int4 *nbr;               // neighbours, -1 = none
    const uint32_t *fan_off;       // [V+1] incident-face list per vertex
    const int2 *fan8;              // [kFanInline][V] its first kFanInline entries, padded with (i, i)
    const int2 *fan;               // (b, c) with face (i, b, c) counter-clockwise
};

struct DevCam {
    int W, H, tiles_x, tiles_y;
    float fx, fy, cx, cy;
    float lb_c1;   // lower bound of the 3-D distance per pixel ring, per metre of depth
};

// DevStats::status set by a kernel: -4 the pose system is not positive
// definite; kStatusBucketOverflow a count found the overflow list full
// (counters not cleared: an internal error).
constexpr int kStatusBucketOverflow = -16;

// Per-iteration bookkeeping written by the kernels and read back per frame.
struct DevStats {
    int n_valid_px, n_assoc_px, n_obs_verts, status;
    float energy[256];
    float step_norm[256];
};

// Offset and normal buffers: SoA x, y, z of V floats each (skinned vertices
// are float4 (x, y, z, 0) so that neighbour gathers are single loads).
struct Vec3Buf { float *x, *y, *z; };

// Fixed-point per-vertex accumulators of the association.
struct Accum {
    uint32_t* cnt;           // pixels per vertex
    long long *sx, *sy, *sz; // sum of (p - v) in units of 2^-32 m
};

// Bucket (index/z-buffer) storage.  Pixels are numbered tile-major (8x8
// tiles in row-major order, 64 pixels per tile in Morton order), so a 4x4
// quadrant of a tile ("cell") is 16 consecutive pixels and pixel k lies in
// cell k >> 4.  Every counted vertex goes straight into its cell's region of
// `cellv`; the regions were laid out by the previous association from the
// counts it read (with room for the surface to move, see layout_tiles), and
// a vertex that finds its cell's region full goes to the overflow list after
// the regions.  The counters are double-buffered: the association reads one
// parity and writes the other's layout (counters cleared), which the next
// count fills.
struct Buckets {
    uint4* cells[2];   // [cells + 1] per parity: (zmin bits, zmax bits, vertices counted, first slot
                       // of the cell's region); entry `cells` holds the end of the last region in .w
    uint32_t* tsum[2]; // [tiles] per parity: vertices counted per tile
    uint32_t* ovfn;    // [2] vertices in the overflow list, per parity
    float4* cellv;     // [ncap + V] (x, y, z, vertex id bits): the cells' regions, then the overflow list
    int ncap;          // slots of the regions (bucket_capacity bounds every layout)
    int4* bstat;       // [tiles] valid, matched, newly observed pixels per tile
    const int* torder; // [ntorder] the tile each association workgroup takes, -1 none (see
                       // tile_order in track.hip: entry k runs on XCD k % 8, each XCD's tiles
                       // nearest the image centre first)
    int ntorder;       // a multiple of 8
    uint32_t* scnt;    // [2][kXcds] per parity: tiles the screen queued for each XCD's search workgroups
    int* tlist;        // [kXcds][capx] the queued tiles
    int capx;          // queue length per XCD (a tile beyond it is searched by its screen wave)
};

// Summary of one frame, written by the frame-end kernel.
struct DevSummary {
    int status, n_valid_px, n_assoc_px, n_obs_verts;
    float energy_first, energy_last, step_norm_last;
    int reason;   // 0 ok, 1 not positive definite, 2 no valid pixel, 3 nothing matched, 4/5 diverged,
                  // 6 bucket index overflow
};

// ---------------------------------------------------------------------------
// Slot table.  Every kernel works on a batch of tracking streams ("slots"):
// its grid is the concatenation of each slot's own grid, and a workgroup finds
// its slot by a binary search of the per-kind workgroup prefix.  A single
// tracker is a batch of one.  The table is rewritten by the host before each
// frame; kernels address the double-buffered vertices and the triple-buffered
// offsets relative to the frame-start indices held in the table, so one
// captured frame serves every starting state.
// ---------------------------------------------------------------------------
constexpr int kSlotBeginFrame = 1;    // the launch starts a frame of this slot
constexpr int kSlotEndFrame = 2;      // the launch ends a frame of this slot
constexpr int kSlotRefreshPose = 4;   // redo forward kinematics at frame start

struct alignas(16) Slot {
    DevModel m;
    DevCam c;
    const JointTable* jt;
    TreeRef tree;                 // tree form of the pose solve
    const uint32_t* anc;          // [L*4] joints on each link's chain
    Buckets b;
    Accum a;
    float* dq;                    // [L*8] link offsets
    float* xi;                    // [P*8] world joint generators
    double *theta, *theta_backup, *step, *gram;
    float* partials;              // [negrid][PP*PP]
    float4* verts[2];
    Vec3Buf normals;
    Vec3Buf phi[3];
    const float* depth;           // frame input: depth image ...
    const float* xyz;             // ... or organised point cloud (the other is null)
    int32_t* assoc;
    DevStats* st;
    DevSummary* summary;
    int PP, negrid, flags;
    float tau, lambda_k, lphi, lnbr, lt, lw;
    int v_cur;                    // current vertex buffer when the launch starts
    int phi_cur, phi_prev;        // current and previous-frame offset buffers
    int iter;                     // iteration of the frame the launch starts at
    int blend;                    // 0 dual-quaternion blend, kBlendLinear: linear blend of the links' motions
    int bpar;                     // bucket counters filled by the next count when the launch starts
};

// Offset buffer written by the step after `src` (never the previous frame's
// buffer, so a failed frame can return to it).
__host__ __device__ __forceinline__ int phi_next(int src, int prev) {
    int n = 0;
    while (n == src || n == prev) ++n;
    return n;
}

// offset buffer current after `n` offset steps of the frame
__host__ __device__ __forceinline__ int phi_index(const Slot& S, int n) {
    int q = S.phi_cur;
    for (int k = 0; k < n; ++k) q = phi_next(q, S.phi_prev);
    return q;
}

enum KernelKind {
    KK_ONE = 0,     // one workgroup per slot (frame bookkeeping, FK, solve)
    KK_VERT,        // ceil(V / 256) workgroups
    KK_CLEAR,       // ceil(max(2 (cells + 1), V) / 256)
    KK_LAYOUT,      // ceil(tiles / kLayoutTiles): bucket layout
    KK_SCREEN,      // one wave per entry of the tile order: the association's screen
    KK_ASSOC,       // association: layout + normals + one search workgroup per entry of the tile order
    KK_ASSOCQ,      // association after a screen: layout + normals + the queued tiles' search workgroups
    KK_NE,          // normal-equation workgroups
    KK_REDUCE,      // Gram reduction workgroups
    KK_VERT64,      // ceil(V / 64): one wave per 64 vertices
    KK_COUNT_
};

struct Batch {
    const Slot* slots;   // [n] device table
    const int* pre;      // [KK_COUNT_][n + 1] exclusive prefix of workgroups per slot
    int n;
};

// host-side launch description: the batch and its grid per kernel kind
struct Launch {
    Batch B;
    int grid[KK_COUNT_];
    int solve_n;        // largest padded pose-system size of the batch
    int solve_elems;    // largest tree-form front storage of the batch; 0: dense form
    int solve_words;    // largest tree-form plan blob of the batch
    int ne_pp, ne_l;    // largest padded Gram size and link count of the batch
    hipStream_t s;
    const Slot* stage_src;   // the window in pinned memory (device view)
    const int* stage_pre;
    // a timed pass: its first kernel stamps t_start and its last kernel
    // t_stop with the kernels' own dispatch timestamps
    hipEvent_t t_start = nullptr, t_stop = nullptr;
};

// Launch `kernel` on L's stream; `first` / `last` mark the kernel's place in
// its pass, so a timed pass's events go to the dispatch packets themselves.
template <typename F, typename... Args>
inline void launch_kernel(const Launch& L, bool first, bool last, F kernel, dim3 grid, dim3 block, uint32_t lds,
                          Args... args) {
    hipEvent_t e0 = first ? L.t_start : nullptr, e1 = last ? L.t_stop : nullptr;
    if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, block, lds, L.s, e0, e1, 0u, args...);
    else hipLaunchKernelGGL(kernel, grid, block, lds, L.s, args...);
}

// n (>= 1) floats from global memory to LDS, every load of a thread issued
// before its first store (a one-wave workgroup copies the link table in one
// round of loads rather than one round per 64 entries)
__device__ __forceinline__ void copy_to_lds(float* dst, const float* __restrict__ src, int n) {
    for (int base = threadIdx.x; base < n; base += 8 * blockDim.x) {
        float t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] = src[min(base + j * (int)blockDim.x, n - 1)];   // past n: not stored
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (base + j * (int)blockDim.x < n) dst[base + j * blockDim.x] = t[j];
    }
}

// Global memory read, written and updated as such.  Through a generic
// pointer the compiler emits flat instructions, which also count as LDS
// accesses: the next wait for LDS (a shuffle, an LDS read, a barrier) or for
// a scalar load then waits for every one of them still in flight.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
__device__ __forceinline__ float4 ldg(const float4* p) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f t = *(const __attribute__((address_space(1))) v4f*)p;
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ int4 ldg(const int4* p) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i t = *(const __attribute__((address_space(1))) v4i*)p;
    return make_int4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ int2 ldg(const int2* p) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    const v2i t = *(const __attribute__((address_space(1))) v2i*)p;
    return make_int2(t.x, t.y);
}
__device__ __forceinline__ uint4 ldg(const uint4* p) {
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const v4u t = *(const __attribute__((address_space(1))) v4u*)p;
    return make_uint4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ uint2 ldg(const uint2* p) {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    const v2u t = *(const __attribute__((address_space(1))) v2u*)p;
    return make_uint2(t.x, t.y);
}
// x, y, z of a float4 (w = 0): an unused fourth register of a load in
// flight would be taken for other values, which must then wait for the load
__device__ __forceinline__ float4 ldg_xyz(const float4* p) {
    typedef float v3f __attribute__((ext_vector_type(3)));
    const v3f t = *(const __attribute__((address_space(1))) v3f*)p;
    return make_float4(t.x, t.y, t.z, 0.0f);
}
template <class T>
__device__ __forceinline__ void stg(T* p, T v) {
    *(__attribute__((address_space(1))) T*)p = v;
}
__device__ __forceinline__ void stg(float4* p, float4 v) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f t;
    t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
    *(__attribute__((address_space(1))) v4f*)p = t;
}
// relaxed device-scope atomics
__device__ __forceinline__ uint32_t atomic_add_g(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add((__attribute__((address_space(1))) uint32_t*)p, v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_add_g(unsigned long long* p, unsigned long long v) {
    return __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long*)p, v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_min_g(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_min((__attribute__((address_space(1))) uint32_t*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_max_g(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_max((__attribute__((address_space(1))) uint32_t*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Keeps a loaded value where it stands: the compiler would otherwise move a
// load into the branch that alone uses it, to be waited for there on its
// own instead of together with the loads issued before it.  Emits nothing.
__device__ __forceinline__ void pin_load(int& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin_load(uint32_t& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin_load(int2& x) { pin_load(x.x); pin_load(x.y); }

// A value the whole wave holds alike (a field of its workgroup's slot), in
// scalar registers: where the compiler cannot tell that it is uniform (a
// value carried through a loop that also copies into LDS) it would keep a
// copy per lane in vector registers.
template <class T>
__device__ __forceinline__ T* wave_uniform(T* p) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float wave_uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// slot of workgroup `blk` of kernel kind `kind`, and its index in that slot
__device__ __forceinline__ int slot_of(const Batch& B, int kind, int blk, int& local) {
    const int* p = B.pre + kind * (B.n + 1);
    int lo = 0, hi = B.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (p[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    local = lo == 0 ? blk : blk - p[lo];  // every prefix starts at 0
    return lo;
}

int ne_grid(int V);

// Association launch: layout workgroups, normal workgroups, then (from a
// multiple of 8, so that workgroup k runs on XCD k % 8) the tiles' search
// workgroups -- one per entry of the tile order (entry k on XCD k % 8), or,
// for a batch of streams, behind a screen launch (one wave per entry of the
// tile order) that finishes the tiles where nothing can match and queues
// the others per XCD, one search workgroup per queue entry
constexpr int kAssocThreads = 512;
constexpr int kXcds = 8;             // workgroups are dealt to the chip's XCDs in turn
constexpr int kLayoutTiles = kAssocThreads;   // tiles per layout workgroup (one per thread)
__host__ __device__ inline int layout_blocks(int ntiles) { return (ntiles + kLayoutTiles - 1) / kLayoutTiles; }
__host__ __device__ inline int assoc_normal_blocks(int V) { return (V + kAssocThreads - 1) / kAssocThreads; }
// the layout and normal workgroups, rounded up to a multiple of kXcds
__host__ __device__ inline int assoc_extra_blocks(int ntiles, int V) {
    return (layout_blocks(ntiles) + assoc_normal_blocks(V) + kXcds - 1) / kXcds * kXcds;
}
// Queue length per XCD: a quarter of the tiles over the XCDs (a body in the
// image leaves most tiles to the screen).
inline int screen_queue(int ntiles) { return std::max(16, (ntiles + 4 * kXcds - 1) / (4 * kXcds)); }

// Slots of the cells' regions.  A layout gives tile t d + d/2 + 32 slots, d
// the largest count of the 3x3 tiles around it; the d sum to about 2 V on a
// body (9 V at most), so 4 V + 32 per tile leaves room to spare.  Regions
// past the end are cut to nothing (their vertices take the overflow list):
// a layout never writes outside the buffer, whatever the counts.
inline int bucket_capacity(int V, int ntiles) { return 4 * V + 32 * ntiles; }

// workgroups of each kind for one slot (host side)
inline int slot_blocks(const Slot& s, int kind) {
    const int V = s.m.V, ntiles = s.c.tiles_x * s.c.tiles_y;
    switch (kind) {
        case KK_ONE: return 1;
        case KK_VERT: return (V + 255) / 256;
        case KK_CLEAR: { const int n = 2 * (4 * ntiles + 1); return ((n > V ? n : V) + 255) / 256; }
        case KK_LAYOUT: return layout_blocks(ntiles);
        case KK_SCREEN: return s.b.ntorder;
        case KK_ASSOC: return assoc_extra_blocks(ntiles, V) + s.b.ntorder;
        case KK_ASSOCQ: return assoc_extra_blocks(ntiles, V) + kXcds * s.b.capx;
        case KK_NE: return s.negrid;
        case KK_REDUCE: { int nb = s.PP >> 4; return nb * (nb + 1) / 2 * 8; }
        case KK_VERT64: return (V + 63) / 64;
    }
    return 0;
}

// ---- launchers (each defined next to its kernels) -------------------------
// vsel: 0 = the slot's vertex buffer at the launch's start, 1 = the other;
// pn: number of offset steps taken so far (see phi_index).
// Which slots take the optional part of a kernel:
enum SlotSel { SEL_NONE = 0, SEL_ALL = 1, SEL_BEGIN = 2, SEL_NOT_END = 3 };
__device__ __forceinline__ bool selected(const Slot& S, int sel) {
    return sel == SEL_ALL || (sel == SEL_BEGIN && (S.flags & kSlotBeginFrame)) ||
           (sel == SEL_NOT_END && !(S.flags & kSlotEndFrame));
}
// copy a table window (slots and prefix rows) from host-visible pinned memory
void launch_stage(hipStream_t s, const Slot* src, Slot* dst, int n, const int* psrc, int* pdst, int npre);
void launch_frame_begin(const Launch& L);
void launch_frame_end(const Launch& L, int first_pose, int last_pose);  // iterations of the frame, -1 = none
void launch_fk(const Launch& L);
// bsel: 0 = the bucket counters of parity Slot::bpar, 1 = the other.
// skin into vsel for the slots selected by `which`; `count` of them also
// enter the buckets of bsel (count_only: the counts alone, for a layout);
// `clear_acc` slots have their accumulators zeroed
void launch_skin(const Launch& L, int vsel, int pn, int which, int count, int bsel, int count_only,
                 int clear_acc);  // count: a SlotSel
void launch_normals(const Launch& L, int vsel);
void launch_clear(const Launch& L);                 // both parities' bucket records (no layout), accumulators,
                                                    // front image
void launch_clear_acc(const Launch& L);             // accumulators only
void launch_clear_counts(const Launch& L, int bsel);  // bsel's counters, its layout kept
void launch_bucket_count(const Launch& L, int vsel, int which, int bsel);
void launch_layout(const Launch& L, int bsel);      // bsel's counts -> the other parity's layout
// association of the surface vsel counted into bsel; the same launch forms
// the surface's normals and lays out the other parity from bsel's counts
// sflip: 1 takes the screen queues of the other parity (repeated launches on
// one parity of the buckets alternate them)
void launch_associate(const Launch& L, int vsel, int bsel, int sflip = 0);
void launch_normal_eq(const Launch& L, int gram_mode, int vsel, int pn);
void launch_gram_reduce(const Launch& L);
void launch_pose_solve(const Launch& L, int fp64, int iter);
bool tree_solve_fits(int elems, int words);   // the tree form's LDS fits the kernel in both precisions
bool prepare_pose_solve();   // once per process, before the first launch
bool prepare_normal_eq();    // likewise
// offset step from v_old / v_new (normals of v_new formed in place); the
// slots selected by `next` also skin the new offsets into v_new ^ 1 and count
// them into the buckets of bsel
void launch_shape(const Launch& L, int fp64, int v_old, int v_new, int pn, int next, int bsel);

}  // namespace trk
