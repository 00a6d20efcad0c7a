/*
 * track.h -- C ABI of the MI355X tracking library (libtrack.so).
 *
 * The library runs the per-frame Gauss-Newton step of the joint skeleton and
 * mesh tracker of Walsman, Wan, Schmidt and Fox, "Dynamic High Resolution
 * Deformable Articulated Tracking" (3DV 2017): dual-quaternion blend
 * skinning of a template mesh (Section 3), projective association of every
 * depth pixel to its nearest skinned vertex, point-to-plane residuals, the
 * pose normal equations and damped Cholesky step (Sections 4.1, 4.2) and the
 * regularised per-vertex offset update (Section 4.3).
 *
 * Conventions for every call:
 *   - Returns TRACK_OK (0) or a negative track_status; nothing is thrown or
 *     aborted across the ABI.  track_last_error() gives a message for the
 *     last failure on the calling thread.
 *   - Input arrays are read during the call only and copied where kept; the
 *     caller keeps ownership.  Output arrays are caller-allocated; a NULL
 *     output pointer means "skip".
 *   - Host pointers unless a flag says the pointer is device memory.
 *   - A context is used from one host thread at a time; contexts are
 *     independent.  Work is issued on the HIP stream given at init (NULL =
 *     the default stream) and calls return when their work has finished.
 *   - Camera frame: +z forward, +y down, metres; pixel centres at integer
 *     (u, v); a point (x, y, z) projects to u = fx*x/z + cx, v = fy*y/z + cy.
 *   - Dual quaternions are stored as 8 numbers (r.w r.x r.y r.z d.w d.x d.y
 *     d.z) for H = r + eps d.
 */
#ifndef TRACK_H
#define TRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct track_ctx track_ctx; /* opaque; owned by the library */

typedef enum {
    TRACK_OK = 0,
    TRACK_E_INVALID = -1, /* bad argument or model; nothing changed            */
    TRACK_E_NOMEM = -2,   /* device allocation failed                           */
    TRACK_E_DEVICE = -3,  /* a HIP call failed                                  */
    TRACK_E_NOT_PD = -4,  /* pose system not positive definite; state kept      */
    TRACK_E_LOST = -5,    /* frame rejected by the health check; state restored */
    TRACK_E_BUDGET = -6   /* would exceed the memory budget                     */
} track_status;

enum { TRACK_HINGE = 0, TRACK_PRISMATIC = 1 };
/* How a vertex's links are combined (Section 3.2): the weighted blend of the
   links' dual quaternions applied to the point (the paper's), or the
   weighted average of the point moved rigidly by each link (matrix linear
   blend skinning). */
enum { TRACK_BLEND_DQ = 0, TRACK_BLEND_LINEAR = 1 };
/* Operand form of the J^T J / J^T r contraction on the matrix cores:
   float32; bfloat16 hi/lo split (3 products); bfloat16 hi/mid/lo split (6). */
enum { TRACK_GRAM_FP32 = 0, TRACK_GRAM_BF16X3 = 1, TRACK_GRAM_BF16X6 = 2 };

/* Compile-time limits of the library. */
#define TRACK_MAX_JOINTS 127
#define TRACK_MAX_LINKS 255
#define TRACK_MAX_INFL 4

/*
 * Template model (Section 3).  The skeleton is a tree of elementary 1-DoF
 * joints, parents listed before children (Section 3.1); a multi-DoF joint is
 * several hinges in succession.  Joint j's frame is
 *     H_{0,j} = H_{0,P(j)} * O_j * H_j(theta_j)
 * with O_j the fixed offset given below and H_j Eq. (1) (hinge) or Eq. (2)
 * (prismatic).  Theta = 0 is the bind pose (Section 3.2).  Each link rides
 * the frame of one joint.  The mesh is V template vertices and F triangles;
 * each vertex has at most TRACK_MAX_INFL (link, weight) pairs whose weights
 * sum to one (Section 3.2).  Neighbours are the four closest template
 * vertices used by the offset regulariser (Section 4.3).
 */
typedef struct {
    int32_t n_joints;            /* P, 1..TRACK_MAX_JOINTS                          */
    const int32_t *joint_parent; /* [P] parent joint, -1 = camera frame; < own index */
    const int32_t *joint_type;   /* [P] TRACK_HINGE or TRACK_PRISMATIC               */
    const float *joint_axis;     /* [P*3] unit axis z in the joint frame             */
    const float *joint_offset;   /* [P*7] O_j: rotation quaternion (w,x,y,z), then
                                    translation (x,y,z); x -> R x + t               */
    int32_t n_links;             /* L, 1..TRACK_MAX_LINKS                            */
    const int32_t *link_joint;   /* [L] joint whose frame the link rides             */
    int32_t n_verts;             /* V >= 1                                           */
    const float *rest_xyz;       /* [V*3] template vertices at Theta = 0             */
    int32_t n_faces;             /* F >= 0                                           */
    const int32_t *faces;        /* [F*3] vertex indices, counter-clockwise seen
                                    from outside (normals point outward)             */
    int32_t max_infl;            /* K, 1..TRACK_MAX_INFL                             */
    const int32_t *skin_link;    /* [V*K] link index or -1 for an unused slot        */
    const float *skin_w;         /* [V*K] weights in [0,1]; sum per vertex within
                                    1e-4 of 1; 0 in unused slots                     */
    const int32_t *neighbors;    /* [V*4] template neighbours (-1 = none) or NULL:
                                    the library takes the 4 nearest template
                                    vertices (ties to the lower index)              */
    float scale;                 /* uniform size of the template (Section 5.4 fits one
                                    such factor per subject from its height), > 0,
                                    1 = as given.  Applied at init about c, the
                                    translation of joint 0's offset: rest vertices
                                    x -> c + s (x - c); offsets of joints with a
                                    parent t -> s t; of other root joints
                                    t -> c + s (t - c).  Prismatic values and the
                                    camera stay in metres.                          */
    int32_t blend;               /* TRACK_BLEND_DQ (0) or TRACK_BLEND_LINEAR           */
} track_model;

/* Pinhole depth camera; depth frames are H x W float32 row-major, metres,
   0 or non-finite = no measurement (Section 4.1). */
typedef struct {
    int32_t width, height; /* 1..4096 each                          */
    float fx, fy, cx, cy;  /* focal lengths (> 0) and principal point */
} track_camera;

/*
 * Tracker constants (Section 4).  One frame runs n_iters iterations; each
 * associates the frame with the current surface and then, as flagged, takes
 * a pose step and/or a per-vertex offset step reusing that association.
 */
typedef struct {
    float tau;                /* association cutoff (m) > 0                          */
    int32_t n_iters;          /* iterations per frame, 1..256                        */
    const uint8_t *do_pose;   /* [n_iters] take the pose step on iteration t         */
    const uint8_t *do_shape;  /* [n_iters] take the offset step on iteration t       */
    float lambda_k;           /* Marquardt damping of the pose step                  */
    float lambda_s;           /* default-pose prior weight (0 = off)                 */
    float lambda_phi;         /* offset magnitude weight                             */
    float lambda_nbr;         /* neighbour smoothness weight                         */
    float lambda_t;           /* temporal weight toward the previous frame's offsets */
    float lambda_w;           /* Marquardt damping of the per-vertex step            */
    int32_t gram_mode;        /* TRACK_GRAM_FP32, _BF16X3 or _BF16X6                  */
    int32_t pose_solve_fp64;  /* 1 = pose Cholesky in float64, 0 = float32           */
    int32_t shape_solve_fp64; /* 1 = per-vertex 3x3 solves in float64                */
    const uint8_t *active;    /* [P] 0 freezes a joint, or NULL = all active         */
} track_params;

typedef struct {
    int32_t status;        /* track_status of the frame                          */
    int32_t n_valid_px;    /* pixels with a measurement                          */
    int32_t n_assoc_px;    /* pixels associated on the last iteration            */
    int32_t n_obs_verts;   /* vertices with at least one pixel, last iteration   */
    float energy_first;    /* sum of squared residuals at the first pose step    */
    float energy_last;     /* the same at the last pose step                     */
    float step_norm_last;  /* |x| of the last pose step                          */
    float ms_total;        /* GPU time of the frame in milliseconds              */
} track_frame_stats;

/*
 * Device memory provider.  alloc returns `bytes` of device memory on the
 * current device, aligned to 256 bytes, or NULL (the call then fails with
 * TRACK_E_NOMEM); free releases what alloc returned.  `user` is passed back
 * unchanged.  A context takes all of its device memory through these calls
 * (one block for the stream's buffers, one for its launch table), at
 * track_init, and returns it at track_destroy, after its stream has drained;
 * nothing is allocated between.  Pinned host memory for the launch table is
 * the library's own.  With no provider the library uses hipMalloc/hipFree.
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} track_allocator;

/*
 * Create a context: validates and copies the model, camera and constants,
 * allocates device memory (through `allocator` if not NULL), and poses the
 * template at theta0 (P doubles: the starting pose the method needs at the
 * head of a sequence, Section 4 opening) with offsets phi0 ([V*3], or NULL
 * for the undeformed template Phi = 0, Section 3.3).  hip_stream is a
 * hipStream_t or NULL.  On success *out holds the context; on failure
 * nothing stays allocated.
 */
int track_init(const track_model *model, const track_camera *camera, const track_params *params,
               const double *theta0, const float *phi0, void *hip_stream, const track_allocator *allocator,
               track_ctx **out);

/*
 * Track one depth frame (H*W float32, metres, row-major; 0 or non-finite =
 * no measurement).  Each pixel's point is back-projected through the camera
 * (Section 4.1), then the iterations of the schedule run: association of
 * every point with its nearest skinned vertex within tau, point-to-plane
 * residuals (Eq. 6), the damped pose step (Eq. 7, 8, Section 4.2) and the
 * per-vertex offset step (Section 4.3).  depth_on_device != 0 means a device
 * pointer, read during the call only; a host frame is copied in.  On success
 * the state holds the new Theta and Phi.  On TRACK_E_NOT_PD or TRACK_E_LOST
 * the state is that of the previous frame.
 */
int track_frame(track_ctx *ctx, const float *depth, int32_t depth_on_device);

/* Same, from an organised point cloud (H*W*3 float32, camera frame; a pixel
   with z <= 0 or a non-finite coordinate has no measurement).  Each pixel's
   point must lie on that pixel's ray, i.e. project onto the pixel's centre
   to within float32 rounding, as the back-projection of a depth image does:
   the nearest-vertex search is bounded by the pixel distance from the
   point's own pixel, so a point placed elsewhere may get a vertex that is
   not its nearest. */
int track_frame_xyz(track_ctx *ctx, const float *xyz, int32_t on_device);

/*
 * track_frame without allocating: for callers that cannot allocate device
 * memory or instantiate graphs while tracking (tight serving loops,
 * harnesses that forbid allocation after set-up).  Same arguments, result
 * and state as track_frame, bit for bit.  The frame's working buffers (bucket
 * index, per-vertex sums, matches, Gram matrices, the pose solve's front
 * image, a staging copy of a host depth image) come from one static block of
 * 64 MiB per GPU instead of the context's memory; the block is held until
 * the process ends and every call on that GPU shares it, so calls that
 * overlap on one GPU race (issue them from one thread, or serialise them).
 * The kernels are launched directly, not from a graph.  TRACK_E_INVALID if
 * the frame's working buffers exceed 64 MiB (about 20 MiB for 50k vertices
 * with 640x480 depth, 108 bytes more per vertex: up to about 440k vertices
 * at that size) or kernel timing is on.  Working buffers read back through
 * track_dbg_get (matches, counts, Gram) are those of track_frame's last frame.
 */
int track_frame_noalloc(track_ctx *ctx, const float *depth, int32_t depth_on_device);

/* Copy the state out: the joint parameters Theta [P] float64 and offsets
   Phi [V*3] that the method estimates per frame (Section 4.1 opening), the
   skinned vertices [V*3] of Eq. (5) at that state, and the last frame's
   statistics.  NULL skips an output.  Never changes the state; waits for the
   context's stream. */
int track_state(const track_ctx *ctx, double *theta, float *phi, float *verts,
                track_frame_stats *stats);

/* Origins of the joint frames at the current Theta (Section 3.1): H_{0,j}
   applied to the origin for every elementary joint j, [P*3] float64, camera
   frame, computed on the host.  A link sits at its joint's origin; this is
   what joint-position accuracy (Section 5.1) is measured on. */
int track_joint_positions(const track_ctx *ctx, double *xyz);

/* Replace the state (checkpoint restore): Theta [P], Phi [V*3] (NULL = 0);
   the previous-frame offsets become Phi as well. */
int track_reset(track_ctx *ctx, const double *theta, const float *phi);

/* Replace the per-frame constants (same model and camera). */
int track_set_params(track_ctx *ctx, const track_params *params);

void track_destroy(track_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *track_last_error(void);

/* ------------------------------------------------------------------------
 * Template refinement (Section 3.3): a low-resolution polygon mesh with skin
 * weights, refined by rounds of Catmull-Clark subdivision into the
 * high-resolution triangle mesh the tracker takes (host computation, once
 * per template).
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_verts;             /* V >= 3                                           */
    const float *xyz;            /* [V*3]                                            */
    int32_t n_faces;             /* F >= 1 polygons, every edge shared by <= 2 faces  */
    const int32_t *face_start;   /* [F+1] face f is face_verts[face_start[f] ..
                                    face_start[f+1]), >= 3 corners, counter-clockwise
                                    seen from outside; face_start[0] = 0            */
    const int32_t *face_verts;
    int32_t max_infl;            /* K >= 1                                           */
    const int32_t *skin_link;    /* [V*K] link or -1                                 */
    const float *skin_w;         /* [V*K]                                            */
} track_polymesh;

/*
 * `levels` (1..4) rounds of Catmull-Clark subdivision: face points are the
 * means of their faces' corners; an interior edge point is the mean of the
 * edge's ends and its two face points, a boundary one the edge's midpoint;
 * an interior vertex of valence n moves to (Q + 2R + (n - 3) S) / n (Q the
 * mean of its face points, R of its edges' midpoints, S its position), a
 * boundary vertex with two boundary edges to (a + b) / 8 + 3 S / 4.  The
 * skin weights are carried through with the same masks (Section 3.3), then
 * each vertex keeps its max_infl_out (1..TRACK_MAX_INFL) largest weights (ties
 * to the lower link) scaled to sum to one.  The final quadrilaterals are
 * split along their shorter diagonal (ties: the one through the first
 * corner) into two counter-clockwise triangles.
 * Numbering per round: vertex points in input order, edge points in order of
 * first appearance (faces in order, each face's edges from its first corner
 * on), face points in face order; face f with corners v_0..v_{k-1} becomes
 * the quadrilaterals (v_i, e(v_i, v_i+1), f, e(v_i-1, v_i)), i = 0..k-1, and
 * quadrilateral q the triangles 2q, 2q + 1.
 * *n_verts_out and *n_tris_out receive the sizes; the array outputs (caller
 * allocated: [V'*3], [T'*3], [V'*max_infl_out] twice) may be NULL, so a first
 * call with NULL arrays sizes them.  TRACK_E_INVALID for an edge with more
 * than two faces or traversed twice in one direction, a face with fewer than
 * three corners, or an index out of range.
 */
int track_subdivide(const track_polymesh *mesh, int32_t levels, int32_t max_infl_out, int32_t *n_verts_out,
                    int32_t *n_tris_out, float *xyz_out, int32_t *tris_out, int32_t *skin_link_out,
                    float *skin_w_out);

/* ------------------------------------------------------------------------
 * Serving: one server tracks many independent streams (each its own model,
 * camera and state, as a context would) under one device-memory budget.
 * Every step runs one Gauss-Newton iteration (Section 4) for every resident
 * stream that has a frame in progress or waiting, in the same kernel
 * launches, so a stream joins at the next iteration boundary after its frame
 * arrives.  A stream's results do not depend on which other streams share
 * its launches.  The server's constants (params) hold for every stream; the
 * per-joint active mask must be NULL.
 * ---------------------------------------------------------------------- */
typedef struct track_server track_server; /* opaque; owned by the library */

typedef struct {
    int32_t stream;          /* id given by track_server_open                    */
    int32_t status;          /* TRACK_OK, TRACK_E_NOT_PD or TRACK_E_LOST          */
    int64_t tag;             /* the caller's tag from track_server_submit         */
    track_frame_stats stats; /* ms_total is 0 (frames share launches)            */
} track_completion;

typedef struct {
    int32_t resident;           /* streams holding device memory                  */
    int32_t waiting;            /* streams queued for admission                   */
    int32_t frames_in_progress; /* frames with iterations still to run            */
    int32_t frames_pending;     /* submitted frames not yet completed             */
    int64_t bytes_used;         /* device bytes of the resident streams           */
    int64_t bytes_budget;
} track_server_stats;

/* Create a server.  hbm_budget_bytes bounds the device memory of resident
   streams; max_streams bounds how many are resident at once (1..4096).
   hip_stream is a hipStream_t or NULL. */
int track_server_create(const track_params *params, int64_t hbm_budget_bytes, int32_t max_streams,
                        void *hip_stream, track_server **out);

/* Open a stream (model, camera and initial state as for track_init).  The
   stream is admitted at once if it fits the budget and the resident count,
   else it waits in arrival order and is admitted when closed streams free
   room; frames may be submitted either way.  TRACK_E_BUDGET if the stream
   alone exceeds the budget.  *stream_id receives its id. */
int track_server_open(track_server *sv, const track_model *model, const track_camera *camera,
                      const double *theta0, const float *phi0, int32_t *stream_id);

/* Queue a depth frame (H*W float32, metres) for a stream; frames of a stream
   are tracked in submission order.  A device frame (on_device != 0) must
   stay valid until its completion is polled; a host frame is copied. */
int track_server_submit(track_server *sv, int32_t stream_id, const float *depth, int32_t on_device,
                        int64_t tag);

/* Admit waiting streams where possible, then run one iteration for every
   resident stream with work; returns when it has finished.  *n_completed
   (may be NULL) receives the number of frames this step completed. */
int track_server_step(track_server *sv, int32_t *n_completed);

/* Move up to max_out completions, oldest first, into out; *n_out receives
   the count. */
int track_server_poll(track_server *sv, track_completion *out, int32_t max_out, int32_t *n_out);

/* Copy a stream's Theta [P] float64 and Phi [V*3] (NULL = skip); not while
   one of its frames is in progress.  A waiting stream reports its initial
   state. */
int track_server_state(track_server *sv, int32_t stream_id, double *theta, float *phi);

/* Close a stream: its device memory returns to the budget and its pending
   frames are dropped without completions. */
int track_server_close(track_server *sv, int32_t stream_id);

int track_server_info(track_server *sv, track_server_stats *out);

void track_server_destroy(track_server *sv);

/* ------------------------------------------------------------------------
 * Per-pass access, for checking each step against an independent
 * implementation on identical inputs.  Buffers are exchanged in the host
 * layouts below; a pass reads and writes the context's buffers.
 * ---------------------------------------------------------------------- */
enum {
    TRACK_BUF_THETA = 0,   /* float64 [P]                                             */
    TRACK_BUF_PHI = 1,     /* float32 [V*3]                                           */
    TRACK_BUF_VERTS = 2,   /* float32 [V*3] skinned vertices of the current surface   */
    TRACK_BUF_NORMALS = 3, /* float32 [V*3] unit vertex normals                       */
    TRACK_BUF_DEPTH = 4,   /* float32 [H*W] (set only)                                */
    TRACK_BUF_XYZ = 5,     /* float32 [H*W*3] (set only)                              */
    TRACK_BUF_ASSOC = 6,   /* int32 [H*W] nearest vertex per pixel or -1 (get only)   */
    TRACK_BUF_COUNT = 7,   /* int32 [V] pixels per vertex                             */
    TRACK_BUF_DELTA = 8,   /* float32 [V*3] mean offset p~_i - v_i (zero if count 0)  */
    TRACK_BUF_GRAM = 9,    /* float64 [(P+1)*(P+1)] [J r]^T [J r], prior excluded (get) */
    TRACK_BUF_STEP = 10,   /* float64 [P] last pose step x (get only)                 */
    TRACK_BUF_PHI_PREV = 11, /* float32 [V*3] previous frame's offsets                */
    TRACK_BUF_VERTS_NEW = 12 /* float32 [V*3] vertices after the pose step (get)     */
};
enum {
    TRACK_PASS_SKIN = 0,      /* FK at THETA, skin PHI -> VERTS, NORMALS                    */
    TRACK_PASS_NORMALS = 1,   /* NORMALS from VERTS                                        */
    TRACK_PASS_ASSOCIATE = 2, /* buckets of VERTS in the layout the last association left
                                 (none after set-up); ASSOC, COUNT, DELTA from the set frame;
                                 NORMALS of VERTS                                            */
    TRACK_PASS_NORMAL_EQ = 3, /* GRAM from THETA, PHI, VERTS, NORMALS, COUNT, DELTA        */
    TRACK_PASS_POSE_STEP = 4, /* damped solve of GRAM; THETA -= x; STEP                    */
    TRACK_PASS_SHAPE = 5      /* re-skin at THETA into VERTS_NEW and new normals, then one
                                 offset step; PHI updated                                  */
};
int track_dbg_set(track_ctx *ctx, int32_t buf, const void *host, size_t bytes);
int track_dbg_get(const track_ctx *ctx, int32_t buf, void *host, size_t bytes);
int track_dbg_run(track_ctx *ctx, int32_t pass);

/* ------------------------------------------------------------------------
 * Kernel timing: when enabled, every launch of the named pass is timed by a
 * pair of HIP events that its first and last kernels stamp from their own
 * dispatch packets on the context's stream (the kernels' execution span);
 * while any timer is on, launches are issued directly, not from graphs.
 * track_kernel_time returns the number of timed launches and their summed
 * duration since the last reset.  The bucket index has no launch of its own
 * inside frames (the kernels that produce a surface count it into the
 * buckets, and the association launch lays them out and forms the normals),
 * so the TRACK_K_BUCKET and TRACK_K_NORMALS timers count no launches.
 * ---------------------------------------------------------------------- */
enum {
    TRACK_K_SKIN = 0,
    TRACK_K_NORMALS = 1,
    TRACK_K_BUCKET = 2,
    TRACK_K_ASSOC = 3,
    TRACK_K_NORMAL_EQ = 4,
    TRACK_K_SOLVE = 5,
    TRACK_K_SHAPE = 6,
    TRACK_K_COUNT_ = 7
};
int track_kernel_timing(track_ctx *ctx, int32_t kernel, int32_t enable);
int track_kernel_time(track_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms);

/* Mean duration of one launch of a pass, from `reps` back-to-back launches on
 * the context's stream between a single pair of HIP events (so the events'
 * own cost is spread over the launches).  Only passes whose repeated launches
 * redo the same work: TRACK_K_SKIN, TRACK_K_ASSOC (reads `depth`, the device
 * image of the last tracked frame, and the buckets that frame left),
 * TRACK_K_NORMAL_EQ (after one association of `depth`) and TRACK_K_SOLVE (the
 * last Gram matrix); other ids give TRACK_E_INVALID, as does an untracked
 * context for the two passes that read `depth`.  reps in 1..100000.  The
 * tracked state is consumed: reset it (track_reset) before tracking again. */
int track_kernel_bench(track_ctx *ctx, int32_t kernel, const float *depth, int32_t reps, double *ms_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* TRACK_H */
