// Host runtime and C ABI of libtrack: model preparation, device memory,
// the per-frame iteration schedule (Section 4) and per-pass access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/track.h"
#include "common.h"

using namespace trk;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(TRACK_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---- host dual-quaternion helpers (float64) for the one-off tables -------
void hq_mul(const double* a, const double* b, double* o) {
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}
void hdq_mul(const double* a, const double* b, double* o) {
    double r[4], d1[4], d2[4];
    hq_mul(a, b, r);
    hq_mul(a, b + 4, d1);
    hq_mul(a + 4, b, d2);
    for (int c = 0; c < 4; ++c) { o[c] = r[c]; o[4 + c] = d1[c] + d2[c]; }
}

// A captured frame: the kernel sequence depends on which ping-pong buffers
// are current when the frame starts, so graphs are cached per starting state.
struct FrameGraph {
    int v0, p0, s0, mode;       // key: vertex buffer, offset buffer, surface valid, input kind
    unsigned tmask;             // key: kernels timed with events inside the graph
    int v1, p1, s1;             // state after the frame
    hipGraphExec_t exec;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> tev;  // (kernel, start/stop)
    hipEvent_t pending[TRACK_K_COUNT_];
};

struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;  // pairs
    size_t used = 0;
    int64_t launches = 0;
    double total_ms = 0.0;
};

}  // namespace

struct track_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int P = 0, L = 0, V = 0, F = 0, K = 0, PP = 0, W = 0, H = 0, npad = 0, ntiles = 0, negrid = 0;
    // constants
    float tau = 0.05f;
    int n_iters = 1;
    std::vector<uint8_t> do_pose, do_shape, active;
    float lambda_k = 0, lambda_s = 0, lambda_phi = 0, lambda_nbr = 0, lambda_t = 0, lambda_w = 0;
    int gram_mode = 0, pose_fp64 = 0, shape_fp64 = 0;
    std::vector<double> prior_S;  // S_k (vertex share per joint)
    // model tables
    JointTable hjt{};
    JointTable* djt = nullptr;
    DevModel dm{};
    DevCam dc{};
    // device memory
    void* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    double *theta = nullptr, *theta_backup = nullptr, *step = nullptr, *gram = nullptr;
    float *dq = nullptr, *xi = nullptr, *partials = nullptr, *depth_buf = nullptr, *xyz_buf = nullptr;
    uint32_t* anc = nullptr;
    Vec3Buf phi[2]{}, phi_prev{}, normals{};
    float4* verts[2]{};
    int phi_cur = 0, v_cur = 0;
    bool surface_valid = false;
    int input_mode = 0;  // 0 depth, 1 xyz (for the per-pass interface)
    Buckets bk{};
    Accum acc{};
    int32_t* assoc = nullptr;
    DevStats* dstats = nullptr;
    DevStats* hstats = nullptr;  // pinned
    double* htheta = nullptr;    // pinned
    int4* hbstat = nullptr;      // pinned, per association workgroup
    int nassoc = 0;              // association workgroups
    track_frame_stats last{};
    hipEvent_t f0 = nullptr, f1 = nullptr;
    KernelTimer timers[TRACK_K_COUNT_];
    bool use_graphs = true;
    std::vector<FrameGraph> graphs;
    FrameGraph* capturing = nullptr;  // graph under construction
    int last_graph = -1;              // graph launched by the last frame, -1 = none
};

namespace {

template <class T>
T* carve(track_ctx* c, size_t n) {
    size_t bytes = (n * sizeof(T) + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(static_cast<char*>(c->arena) + c->arena_used);
    c->arena_used += bytes;
    return p;
}

void drop_graphs(track_ctx* c);

void timed_begin(track_ctx* c, int k) {
    KernelTimer& t = c->timers[k];
    if (!t.on) return;
    if (c->capturing) {  // events of a captured frame belong to its graph
        hipEvent_t e;
        if (hipEventCreate(&e) == hipSuccess && hipEventRecord(e, c->stream) == hipSuccess) c->capturing->pending[k] = e;
        else c->capturing->pending[k] = nullptr;
        return;
    }
    if (t.used + 2 > t.ev.size()) {
        for (int q = 0; q < 64; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) == hipSuccess) t.ev.push_back(e);
        }
    }
    if (t.used + 2 <= t.ev.size()) (void)hipEventRecord(t.ev[t.used], c->stream);
}
void timed_end(track_ctx* c, int k) {
    KernelTimer& t = c->timers[k];
    if (!t.on) return;
    if (c->capturing) {
        hipEvent_t e;
        hipEvent_t b = c->capturing->pending[k];
        if (b && hipEventCreate(&e) == hipSuccess && hipEventRecord(e, c->stream) == hipSuccess)
            c->capturing->tev.push_back({k, {b, e}});
        return;
    }
    if (t.used + 2 > t.ev.size()) return;
    (void)hipEventRecord(t.ev[t.used + 1], c->stream);
    t.used += 2;
}
// called after a stream synchronisation: fold the recorded pairs into totals
void timed_collect(track_ctx* c) {
    for (auto& t : c->timers) {
        for (size_t q = 0; q + 1 < t.used; q += 2) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, t.ev[q], t.ev[q + 1]) == hipSuccess) {
                t.total_ms += ms;
                t.launches += 1;
            }
        }
        t.used = 0;
    }
    if (c->last_graph >= 0) {
        for (auto& te : c->graphs[c->last_graph].tev) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, te.second.first, te.second.second) == hipSuccess) {
                c->timers[te.first].total_ms += ms;
                c->timers[te.first].launches += 1;
            }
        }
        c->last_graph = -1;
    }
}

// 4 nearest template vertices (ties: lower index) through a uniform grid
std::vector<int> nearest4(const float* xyz, int V) {
    std::vector<int> out(4 * (size_t)V, -1);
    if (V <= 1) return out;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < V; ++i)
        for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], (double)xyz[3 * i + d]); hi[d] = std::max(hi[d], (double)xyz[3 * i + d]); }
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= std::max(hi[d] - lo[d], 1e-6);
    double h = std::cbrt(vol / V) * 1.5;
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = std::max(1, std::min(1024, (int)((hi[d] - lo[d]) / h) + 1));
    auto cell = [&](int d, double x) { return std::min(n[d] - 1, std::max(0, (int)((x - lo[d]) / h))); };
    std::vector<std::vector<int>> grid((size_t)n[0] * n[1] * n[2]);
    for (int i = 0; i < V; ++i)
        grid[((size_t)cell(0, xyz[3 * i]) * n[1] + cell(1, xyz[3 * i + 1])) * n[2] + cell(2, xyz[3 * i + 2])].push_back(i);
    for (int i = 0; i < V; ++i) {
        int c0 = cell(0, xyz[3 * i]), c1 = cell(1, xyz[3 * i + 1]), c2 = cell(2, xyz[3 * i + 2]);
        std::vector<std::pair<double, int>> cand;
        for (int r = 0;; ++r) {
            for (int a = c0 - r; a <= c0 + r; ++a)
                for (int b = c1 - r; b <= c1 + r; ++b)
                    for (int e = c2 - r; e <= c2 + r; ++e) {
                        if (std::max({std::abs(a - c0), std::abs(b - c1), std::abs(e - c2)}) != r) continue;
                        if (a < 0 || b < 0 || e < 0 || a >= n[0] || b >= n[1] || e >= n[2]) continue;
                        for (int j : grid[((size_t)a * n[1] + b) * n[2] + e]) {
                            if (j == i) continue;
                            double dx = (double)xyz[3 * j] - xyz[3 * i], dy = (double)xyz[3 * j + 1] - xyz[3 * i + 1],
                                   dz = (double)xyz[3 * j + 2] - xyz[3 * i + 2];
                            cand.push_back({(dx * dx + dy * dy) + dz * dz, j});
                        }
                    }
            bool all = r >= std::max({n[0], n[1], n[2]});
            if ((int)cand.size() >= 4 || all) {
                std::sort(cand.begin(), cand.end());
                // every vertex closer than r*h has been seen
                if (all || cand[3].first <= (r * h) * (r * h)) break;
            }
        }
        for (int q = 0; q < 4 && q < (int)cand.size(); ++q) out[4 * (size_t)i + q] = cand[q].second;
    }
    return out;
}

int set_params(track_ctx* c, const track_params* p) {
    if (!p) return fail(TRACK_E_INVALID, "params is NULL");
    if (!(p->tau > 0.0f) || !std::isfinite(p->tau)) return fail(TRACK_E_INVALID, "tau must be > 0");
    if (p->n_iters < 1 || p->n_iters > 256) return fail(TRACK_E_INVALID, "n_iters must be in 1..256");
    if (!p->do_pose || !p->do_shape) return fail(TRACK_E_INVALID, "do_pose/do_shape are required");
    if (p->gram_mode != TRACK_GRAM_FP32 && p->gram_mode != TRACK_GRAM_BF16X3 && p->gram_mode != TRACK_GRAM_BF16X6)
        return fail(TRACK_E_INVALID, "unknown gram_mode");
    const float lam[6] = {p->lambda_k, p->lambda_s, p->lambda_phi, p->lambda_nbr, p->lambda_t, p->lambda_w};
    for (float l : lam)
        if (!(l >= 0.0f) || !std::isfinite(l)) return fail(TRACK_E_INVALID, "weights must be finite and >= 0");
    c->tau = p->tau;
    c->n_iters = p->n_iters;
    c->do_pose.assign(p->do_pose, p->do_pose + p->n_iters);
    c->do_shape.assign(p->do_shape, p->do_shape + p->n_iters);
    c->active.assign(c->P, 1);
    if (p->active) c->active.assign(p->active, p->active + c->P);
    c->lambda_k = p->lambda_k; c->lambda_s = p->lambda_s; c->lambda_phi = p->lambda_phi;
    c->lambda_nbr = p->lambda_nbr; c->lambda_t = p->lambda_t; c->lambda_w = p->lambda_w;
    c->gram_mode = p->gram_mode;
    drop_graphs(c);
    c->pose_fp64 = p->pose_solve_fp64 ? 1 : 0;
    c->shape_fp64 = p->shape_solve_fp64 ? 1 : 0;
    for (int k = 0; k < c->P; ++k) {
        double w = (double)c->lambda_s * c->prior_S[k];
        c->hjt.prior[k] = w * w;
        c->hjt.active[k] = c->active[k] ? 1 : 0;
    }
    if (c->djt) HIP_TRY(hipMemcpy(c->djt, &c->hjt, sizeof(JointTable), hipMemcpyHostToDevice));
    return TRACK_OK;
}

int validate_model(const track_model* m, const track_camera* cam) {
    if (!m || !cam) return fail(TRACK_E_INVALID, "model/camera is NULL");
    if (m->n_joints < 1 || m->n_joints > TRACK_MAX_JOINTS) return fail(TRACK_E_INVALID, "n_joints out of range");
    if (m->n_links < 1 || m->n_links > TRACK_MAX_LINKS) return fail(TRACK_E_INVALID, "n_links out of range");
    if (m->n_verts < 1) return fail(TRACK_E_INVALID, "n_verts must be >= 1");
    if (m->n_faces < 0) return fail(TRACK_E_INVALID, "n_faces must be >= 0");
    if (m->max_infl < 1 || m->max_infl > TRACK_MAX_INFL) return fail(TRACK_E_INVALID, "max_infl out of range");
    if (!m->joint_parent || !m->joint_type || !m->joint_axis || !m->joint_offset || !m->link_joint ||
        !m->rest_xyz || (m->n_faces > 0 && !m->faces) || !m->skin_link || !m->skin_w)
        return fail(TRACK_E_INVALID, "missing model array");
    for (int j = 0; j < m->n_joints; ++j) {
        if (m->joint_parent[j] < -1 || m->joint_parent[j] >= j)
            return fail(TRACK_E_INVALID, "joints must be listed parents first");
        if (m->joint_type[j] != TRACK_HINGE && m->joint_type[j] != TRACK_PRISMATIC)
            return fail(TRACK_E_INVALID, "unknown joint type");
        const float* a = m->joint_axis + 3 * j;
        double n = std::sqrt((double)a[0] * a[0] + (double)a[1] * a[1] + (double)a[2] * a[2]);
        if (!(std::fabs(n - 1.0) < 1e-3)) return fail(TRACK_E_INVALID, "joint axis must be unit length");
        const float* o = m->joint_offset + 7 * j;
        double qn = std::sqrt((double)o[0] * o[0] + (double)o[1] * o[1] + (double)o[2] * o[2] + (double)o[3] * o[3]);
        if (!(std::fabs(qn - 1.0) < 1e-3)) return fail(TRACK_E_INVALID, "offset quaternion must be unit length");
        for (int q = 4; q < 7; ++q)
            if (!std::isfinite(o[q])) return fail(TRACK_E_INVALID, "offset translation not finite");
    }
    for (int l = 0; l < m->n_links; ++l)
        if (m->link_joint[l] < 0 || m->link_joint[l] >= m->n_joints) return fail(TRACK_E_INVALID, "link_joint out of range");
    for (int64_t q = 0; q < 3 * (int64_t)m->n_verts; ++q)
        if (!std::isfinite(m->rest_xyz[q])) return fail(TRACK_E_INVALID, "rest_xyz not finite");
    for (int64_t q = 0; q < 3 * (int64_t)m->n_faces; ++q)
        if (m->faces[q] < 0 || m->faces[q] >= m->n_verts) return fail(TRACK_E_INVALID, "face index out of range");
    for (int i = 0; i < m->n_verts; ++i) {
        double s = 0.0;
        int cnt = 0;
        for (int k = 0; k < m->max_infl; ++k) {
            int l = m->skin_link[i * m->max_infl + k];
            float w = m->skin_w[i * m->max_infl + k];
            if (l < -1 || l >= m->n_links) return fail(TRACK_E_INVALID, "skin_link out of range");
            if (!(w >= 0.0f && w <= 1.0f)) return fail(TRACK_E_INVALID, "skin weight outside [0,1]");
            if (l >= 0) { s += w; ++cnt; }
        }
        if (cnt == 0 || !(std::fabs(s - 1.0) <= 1e-4)) return fail(TRACK_E_INVALID, "skin weights must sum to 1");
    }
    if (m->neighbors)
        for (int64_t q = 0; q < 4 * (int64_t)m->n_verts; ++q)
            if (m->neighbors[q] < -1 || m->neighbors[q] >= m->n_verts) return fail(TRACK_E_INVALID, "neighbor out of range");
    if (cam->width < 1 || cam->height < 1 || cam->width > 4096 || cam->height > 4096)
        return fail(TRACK_E_INVALID, "image size out of range");
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !std::isfinite(cam->fx) || !std::isfinite(cam->fy) ||
        !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
        return fail(TRACK_E_INVALID, "bad camera intrinsics");
    return TRACK_OK;
}

void build_joint_table(track_ctx* c, const track_model* m) {
    JointTable& t = c->hjt;
    std::memset(&t, 0, sizeof(t));
    t.P = m->n_joints;
    t.L = m->n_links;
    std::vector<double> H0(8 * (size_t)t.P);
    for (int j = 0; j < t.P; ++j) {
        t.parent[j] = m->joint_parent[j];
        t.type[j] = m->joint_type[j];
        for (int d = 0; d < 3; ++d) t.axis[j][d] = m->joint_axis[3 * j + d];
        const float* o = m->joint_offset + 7 * j;
        double qn = std::sqrt((double)o[0] * o[0] + (double)o[1] * o[1] + (double)o[2] * o[2] + (double)o[3] * o[3]);
        double r[4] = {o[0] / qn, o[1] / qn, o[2] / qn, o[3] / qn};
        double tq[4] = {0.0, 0.5 * o[4], 0.5 * o[5], 0.5 * o[6]};
        double d[4];
        hq_mul(tq, r, d);
        for (int q = 0; q < 4; ++q) { t.off[j][q] = r[q]; t.off[j][4 + q] = d[q]; }
        // bind pose: Theta = 0 makes every H_j the identity
        if (t.parent[j] < 0) std::memcpy(&H0[8 * j], t.off[j], 8 * sizeof(double));
        else hdq_mul(&H0[8 * t.parent[j]], t.off[j], &H0[8 * j]);
    }
    for (int l = 0; l < t.L; ++l) {
        int j = m->link_joint[l];
        t.link_joint[l] = j;
        const double* h = &H0[8 * j];
        double inv[8] = {h[0], -h[1], -h[2], -h[3], h[4], -h[5], -h[6], -h[7]};
        std::memcpy(t.binv[l], inv, sizeof(inv));
        for (int k = j; k >= 0; k = t.parent[k]) t.anc[l][k >> 5] |= 1u << (k & 31);
    }
    // default-pose prior weights: share of vertices with weight on a link
    // whose chain holds joint k; zero for the joints carrying the root link
    c->prior_S.assign(t.P, 0.0);
    std::vector<int> cnt(t.P, 0);
    for (int i = 0; i < m->n_verts; ++i) {
        uint32_t mask[4] = {0, 0, 0, 0};
        for (int k = 0; k < m->max_infl; ++k) {
            int l = m->skin_link[i * m->max_infl + k];
            if (l >= 0 && m->skin_w[i * m->max_infl + k] > 0.0f)
                for (int q = 0; q < 4; ++q) mask[q] |= t.anc[l][q];
        }
        for (int k = 0; k < t.P; ++k) cnt[k] += (mask[k >> 5] >> (k & 31)) & 1u;
    }
    for (int k = 0; k < t.P; ++k) {
        bool root = (t.anc[0][k >> 5] >> (k & 31)) & 1u;
        c->prior_S[k] = root ? 0.0 : (double)cnt[k] / (double)m->n_verts;
    }
}

// --------------------------------------------------------------------------
// the iteration schedule of one frame
// --------------------------------------------------------------------------
void ensure_surface(track_ctx* c) {
    if (c->surface_valid) return;
    timed_begin(c, TRACK_K_SKIN);
    launch_skin(c->stream, c->dm, c->dq, cview(c->phi[c->phi_cur]), c->verts[c->v_cur]);
    timed_end(c, TRACK_K_SKIN);
    timed_begin(c, TRACK_K_NORMALS);
    launch_normals(c->stream, c->dm, c->verts[c->v_cur], c->normals);
    timed_end(c, TRACK_K_NORMALS);
    c->surface_valid = true;
}

void pass_associate(track_ctx* c, const float* depth, const float* xyz) {
    timed_begin(c, TRACK_K_BUCKET);
    launch_clear(c->stream, c->npad, c->bk, c->V, c->acc, c->dstats);
    launch_bucket(c->stream, c->dc, c->V, c->verts[c->v_cur], c->bk);
    timed_end(c, TRACK_K_BUCKET);
    timed_begin(c, TRACK_K_ASSOC);
    launch_associate(c->stream, c->dc, c->tau, depth, xyz, c->bk, c->acc, c->verts[c->v_cur], c->assoc);
    timed_end(c, TRACK_K_ASSOC);
}

void pass_normal_eq(track_ctx* c) {
    timed_begin(c, TRACK_K_NORMAL_EQ);
    launch_normal_eq(c->stream, c->dm, c->PP, c->gram_mode, c->dq, c->xi, c->anc, c->verts[c->v_cur],
                     cview(c->normals), cview(c->phi[c->phi_cur]), c->acc, c->partials, c->negrid);
    timed_end(c, TRACK_K_NORMAL_EQ);
    launch_gram_reduce(c->stream, c->PP, c->negrid, c->partials, c->gram);
}

void pass_pose_step(track_ctx* c, int iter) {
    timed_begin(c, TRACK_K_SOLVE);
    launch_pose_solve(c->stream, c->djt, c->PP, c->gram, c->lambda_k, c->pose_fp64, c->theta, c->step,
                      c->dstats, iter, c->dq, c->xi);
    timed_end(c, TRACK_K_SOLVE);
}

// re-skin at the current pose into the other vertex buffer, then one offset
// step; afterwards that buffer is the current surface
void pass_shape(track_ctx* c, bool reskin) {
    int vo = c->v_cur, vn = c->v_cur;
    if (reskin) {
        vn = c->v_cur ^ 1;
        timed_begin(c, TRACK_K_SKIN);
        launch_skin(c->stream, c->dm, c->dq, cview(c->phi[c->phi_cur]), c->verts[vn]);
        timed_end(c, TRACK_K_SKIN);
        timed_begin(c, TRACK_K_NORMALS);
        launch_normals(c->stream, c->dm, c->verts[vn], c->normals);
        timed_end(c, TRACK_K_NORMALS);
    }
    timed_begin(c, TRACK_K_SHAPE);
    launch_shape(c->stream, c->dm, c->dq, c->verts[vo], c->verts[vn], cview(c->normals), c->acc,
                 cview(c->phi[c->phi_cur]), cview(c->phi_prev), c->phi[c->phi_cur ^ 1], c->lambda_phi,
                 c->lambda_nbr, c->lambda_t, c->lambda_w, c->shape_fp64);
    timed_end(c, TRACK_K_SHAPE);
    c->phi_cur ^= 1;
    c->v_cur = vn;
    c->surface_valid = false;
}

void drop_graphs(track_ctx* c) {
    for (auto& g : c->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        for (auto& te : g.tev) { (void)hipEventDestroy(te.second.first); (void)hipEventDestroy(te.second.second); }
    }
    c->graphs.clear();
    c->last_graph = -1;
}

unsigned timing_mask(const track_ctx* c) {
    unsigned m = 0;
    for (int k = 0; k < TRACK_K_COUNT_; ++k)
        if (c->timers[k].on) m |= 1u << k;
    return m;
}

// the kernels of one frame, issued on the context's stream
void enqueue_frame(track_ctx* c, const float* depth, const float* xyz) {
    launch_frame_begin(c->stream, c->P, c->theta, c->theta_backup, c->dstats);
    for (int t = 0; t < c->n_iters; ++t) {
        ensure_surface(c);
        pass_associate(c, depth, xyz);
        if (c->do_pose[t]) {
            pass_normal_eq(c);
            pass_pose_step(c, t);
        }
        if (c->do_shape[t]) {
            pass_shape(c, c->do_pose[t] != 0);
        } else if (c->do_pose[t]) {
            // re-skin at the new pose; the surface is current again
            c->v_cur ^= 1;
            c->surface_valid = false;
            ensure_surface(c);
        }
    }
}

// Issue one frame as a replay of a cached graph (the frame reads its input
// from the context's own buffer); timing events, when enabled, are part of
// the graph.  If capture is unavailable the kernels are launched directly.
int launch_frame(track_ctx* c, const float* depth, const float* xyz) {
    if (!c->use_graphs) {
        enqueue_frame(c, depth, xyz);
        return TRACK_OK;
    }
    const int mode = xyz ? 1 : 0;
    const float* in = xyz ? xyz : depth;
    float* buf = xyz ? c->xyz_buf : c->depth_buf;
    const size_t bytes = sizeof(float) * (size_t)c->W * c->H * (xyz ? 3 : 1);
    if (in != buf) HIP_TRY(hipMemcpyAsync(buf, in, bytes, hipMemcpyDeviceToDevice, c->stream));
    const int s0 = c->surface_valid ? 1 : 0;
    const unsigned tm = timing_mask(c);
    for (size_t q = 0; q < c->graphs.size(); ++q) {
        FrameGraph& g = c->graphs[q];
        if (g.v0 == c->v_cur && g.p0 == c->phi_cur && g.s0 == s0 && g.mode == mode && g.tmask == tm) {
            HIP_TRY(hipGraphLaunch(g.exec, c->stream));
            c->v_cur = g.v1; c->phi_cur = g.p1; c->surface_valid = g.s1 != 0;
            c->last_graph = (int)q;
            return TRACK_OK;
        }
    }
    FrameGraph g{c->v_cur, c->phi_cur, s0, mode, tm, 0, 0, 0, nullptr, {}, {}};
    const int v0 = c->v_cur, p0 = c->phi_cur;
    const bool sv0 = c->surface_valid;
    hipGraph_t graph = nullptr;
    c->capturing = &g;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue_frame(c, xyz ? nullptr : c->depth_buf, xyz ? c->xyz_buf : nullptr);
        e = hipStreamEndCapture(c->stream, &graph);
    }
    c->capturing = nullptr;
    if (e == hipSuccess) {
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
    }
    if (e != hipSuccess) {
        // no graphs on this stream: restore the state and launch directly
        (void)hipGetLastError();
        for (auto& te : g.tev) { (void)hipEventDestroy(te.second.first); (void)hipEventDestroy(te.second.second); }
        c->v_cur = v0; c->phi_cur = p0; c->surface_valid = sv0;
        c->use_graphs = false;
        enqueue_frame(c, depth, xyz);
        return TRACK_OK;
    }
    g.v1 = c->v_cur; g.p1 = c->phi_cur; g.s1 = c->surface_valid ? 1 : 0;
    c->graphs.push_back(g);
    c->last_graph = (int)c->graphs.size() - 1;
    HIP_TRY(hipGraphLaunch(c->graphs.back().exec, c->stream));
    return TRACK_OK;
}

int run_frame(track_ctx* c, const float* depth, const float* xyz) {
    HIP_TRY(hipEventRecord(c->f0, c->stream));
    int rc = launch_frame(c, depth, xyz);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(c->f1, c->stream));
    HIP_TRY(hipMemcpyAsync(c->hstats, c->dstats, sizeof(DevStats), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->hbstat, c->bk.bstat, sizeof(int4) * c->nassoc, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->htheta, c->theta, sizeof(double) * c->P, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    timed_collect(c);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, c->f0, c->f1);
    DevStats& s = *c->hstats;
    // counts of the last association, summed over its workgroups
    s.n_valid_px = s.n_assoc_px = s.n_obs_verts = 0;
    for (int q = 0; q < c->nassoc; ++q) {
        s.n_valid_px += c->hbstat[q].x;
        s.n_assoc_px += c->hbstat[q].y;
        s.n_obs_verts += c->hbstat[q].z;
    }
    track_frame_stats fs{};
    fs.n_valid_px = s.n_valid_px;
    fs.n_assoc_px = s.n_assoc_px;
    fs.n_obs_verts = s.n_obs_verts;
    int first = -1, lastp = -1;
    for (int t = 0; t < c->n_iters; ++t)
        if (c->do_pose[t]) { if (first < 0) first = t; lastp = t; }
    fs.energy_first = first >= 0 ? s.energy[first] : 0.0f;
    fs.energy_last = lastp >= 0 ? s.energy[lastp] : 0.0f;
    fs.step_norm_last = lastp >= 0 ? s.step_norm[lastp] : 0.0f;
    fs.ms_total = ms;
    // health check: solver failure, nothing measured, nothing matched, or a
    // non-finite pose; the previous frame's state is restored
    int status = TRACK_OK;
    std::string why;
    if (s.status == TRACK_E_NOT_PD) { status = TRACK_E_NOT_PD; why = "pose system not positive definite"; }
    else if (s.n_valid_px == 0) { status = TRACK_E_LOST; why = "frame has no valid pixels"; }
    else if (s.n_assoc_px == 0) { status = TRACK_E_LOST; why = "no pixel matched the surface"; }
    else {
        for (int k = 0; k < c->P; ++k)
            if (!std::isfinite(c->htheta[k])) { status = TRACK_E_LOST; why = "pose diverged"; break; }
        if (!std::isfinite(fs.energy_last)) { status = TRACK_E_LOST; why = "energy diverged"; }
    }
    fs.status = status;
    c->last = fs;
    if (status == TRACK_OK) {
        launch_copy3(c->stream, c->V, cview(c->phi[c->phi_cur]), c->phi_prev);
    } else {
        HIP_TRY(hipMemcpyAsync(c->theta, c->theta_backup, sizeof(double) * c->P, hipMemcpyDeviceToDevice, c->stream));
        launch_copy3(c->stream, c->V, cview(c->phi_prev), c->phi[c->phi_cur]);
        launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
        c->surface_valid = false;
        ensure_surface(c);
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (status != TRACK_OK) return fail(status, why);
    return TRACK_OK;
}

int upload_soa(track_ctx* c, Vec3Buf dst, const float* aos) {
    std::vector<float> t(3 * (size_t)c->V);
    for (int i = 0; i < c->V; ++i) { t[i] = aos[3 * i]; t[c->V + i] = aos[3 * i + 1]; t[2 * c->V + i] = aos[3 * i + 2]; }
    HIP_TRY(hipMemcpy(dst.x, t.data(), sizeof(float) * c->V, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dst.y, t.data() + c->V, sizeof(float) * c->V, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dst.z, t.data() + 2 * c->V, sizeof(float) * c->V, hipMemcpyHostToDevice));
    return TRACK_OK;
}

int download_soa(const track_ctx* c, Vec3Buf src, float* aos) {
    std::vector<float> t(3 * (size_t)c->V);
    HIP_TRY(hipMemcpy(t.data(), src.x, sizeof(float) * c->V, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t.data() + c->V, src.y, sizeof(float) * c->V, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t.data() + 2 * c->V, src.z, sizeof(float) * c->V, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->V; ++i) { aos[3 * i] = t[i]; aos[3 * i + 1] = t[c->V + i]; aos[3 * i + 2] = t[2 * c->V + i]; }
    return TRACK_OK;
}

int upload_v4(track_ctx* c, float4* dst, const float* aos) {
    std::vector<float4> t(c->V);
    for (int i = 0; i < c->V; ++i) t[i] = make_float4(aos[3 * i], aos[3 * i + 1], aos[3 * i + 2], 0.0f);
    HIP_TRY(hipMemcpy(dst, t.data(), sizeof(float4) * c->V, hipMemcpyHostToDevice));
    return TRACK_OK;
}

int download_v4(const track_ctx* c, const float4* src, float* aos) {
    std::vector<float4> t(c->V);
    HIP_TRY(hipMemcpy(t.data(), src, sizeof(float4) * c->V, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->V; ++i) { aos[3 * i] = t[i].x; aos[3 * i + 1] = t[i].y; aos[3 * i + 2] = t[i].z; }
    return TRACK_OK;
}

void free_ctx(track_ctx* c) {
    if (!c) return;
    drop_graphs(c);
    for (auto& t : c->timers)
        for (auto e : t.ev) (void)hipEventDestroy(e);
    if (c->f0) (void)hipEventDestroy(c->f0);
    if (c->f1) (void)hipEventDestroy(c->f1);
    if (c->arena) (void)hipFree(c->arena);
    if (c->djt) (void)hipFree(c->djt);
    if (c->hstats) (void)hipHostFree(c->hstats);
    if (c->htheta) (void)hipHostFree(c->htheta);
    if (c->hbstat) (void)hipHostFree(c->hbstat);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* track_last_error(void) { return g_err.c_str(); }

int track_init(const track_model* model, const track_camera* camera, const track_params* params,
               const double* theta0, const float* phi0, void* hip_stream, track_ctx** out) {
    g_err.clear();
    if (!out) return fail(TRACK_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = validate_model(model, camera);
    if (rc) return rc;
    if (!theta0) return fail(TRACK_E_INVALID, "theta0 is NULL");
    for (int k = 0; k < model->n_joints; ++k)
        if (!std::isfinite(theta0[k])) return fail(TRACK_E_INVALID, "theta0 not finite");
    track_ctx* c = new track_ctx();
    c->P = model->n_joints; c->L = model->n_links; c->V = model->n_verts; c->F = model->n_faces;
    c->K = model->max_infl;
    c->PP = ((c->P + 1) + 15) / 16 * 16;
    c->W = camera->width; c->H = camera->height;
    int tx = (c->W + 7) / 8, ty = (c->H + 7) / 8;
    c->ntiles = tx * ty;
    c->npad = c->ntiles * 64;
    c->negrid = ne_grid(c->V);
    {
        const char* env = std::getenv("TRACK_NO_GRAPH");
        c->use_graphs = !(env && env[0] == '1');
    }
    build_joint_table(c, model);
    if ((rc = set_params(c, params))) { free_ctx(c); return rc; }
    if (hipGetDevice(&c->device) != hipSuccess) { free_ctx(c); return fail(TRACK_E_DEVICE, "no HIP device"); }
    if (hip_stream) c->stream = (hipStream_t)hip_stream;
    else {
        if (hipStreamCreate(&c->stream) != hipSuccess) { free_ctx(c); return fail(TRACK_E_DEVICE, "stream"); }
        c->own_stream = true;
    }
    // ---- device memory (one arena) ----
    const size_t V = c->V, N = (size_t)c->W * c->H;
    size_t need = 0;
    auto add = [&](size_t n, size_t sz) { need += (n * sz + 255) & ~size_t(255); };
    add(c->P, 8); add(c->P, 8); add(c->P, 8); add((size_t)c->PP * c->PP, 8);   // theta, backup, step, gram
    add(8 * c->L, 4); add(8 * c->P, 4); add(4 * c->L, 4);                       // dq, xi, anc
    add((size_t)c->negrid * c->PP * c->PP, 4);                                  // partials
    add(N, 4); add(3 * N, 4);                                                   // depth, xyz
    for (int q = 0; q < 3 * 5; ++q) add(V, 4);                                  // rest, phi x2, prev, normals
    add(V, 16); add(V, 16);                                                     // vertices x2
    add(V, 16); add(V, 4); add(V, 16); add(V + 1, 4); add(3 * (size_t)c->F, 8); // w, links, nbr, fan
    add(c->npad, 4); add(c->npad, 4); add(c->npad, 4); add(c->npad, 16);       // buckets
    add(c->ntiles, 4); add(c->ntiles, 4); add(c->ntiles, 8);
    add(V, 4); add(V, 4); add(V, 16);
    c->nassoc = assoc_blocks(tx, ty);
    add(c->nassoc, 16);
    add(4 * (size_t)c->ntiles, 16);
    add(V, 4); add(V, 8); add(V, 8); add(V, 8);                                 // accumulators
    add(N, 4); add(1, sizeof(DevStats));
    c->arena_bytes = need;
    if (hipMalloc(&c->arena, need) != hipSuccess) { free_ctx(c); return fail(TRACK_E_NOMEM, "device allocation failed"); }
    if (hipMalloc(&c->djt, sizeof(JointTable)) != hipSuccess) { free_ctx(c); return fail(TRACK_E_NOMEM, "device allocation failed"); }
    if (hipHostMalloc(&c->hstats, sizeof(DevStats)) != hipSuccess ||
        hipHostMalloc(&c->htheta, sizeof(double) * c->P) != hipSuccess ||
        hipHostMalloc(&c->hbstat, sizeof(int4) * c->nassoc) != hipSuccess) {
        free_ctx(c);
        return fail(TRACK_E_NOMEM, "pinned allocation failed");
    }
    c->theta = carve<double>(c, c->P);
    c->theta_backup = carve<double>(c, c->P);
    c->step = carve<double>(c, c->P);
    c->gram = carve<double>(c, (size_t)c->PP * c->PP);
    c->dq = carve<float>(c, 8 * c->L);
    c->xi = carve<float>(c, 8 * c->P);
    c->anc = carve<uint32_t>(c, 4 * c->L);
    c->partials = carve<float>(c, (size_t)c->negrid * c->PP * c->PP);
    c->depth_buf = carve<float>(c, N);
    c->xyz_buf = carve<float>(c, 3 * N);
    auto v3 = [&]() { Vec3Buf b; b.x = carve<float>(c, V); b.y = carve<float>(c, V); b.z = carve<float>(c, V); return b; };
    Vec3Buf rest = v3();
    c->phi[0] = v3(); c->phi[1] = v3(); c->phi_prev = v3();
    c->verts[0] = carve<float4>(c, V); c->verts[1] = carve<float4>(c, V); c->normals = v3();
    float4* w4 = carve<float4>(c, V);
    uint32_t* lk = carve<uint32_t>(c, V);
    int4* nb = carve<int4>(c, V);
    uint32_t* fan_off = carve<uint32_t>(c, V + 1);
    int2* fan = carve<int2>(c, 3 * (size_t)c->F);
    c->bk.pcnt = carve<uint32_t>(c, c->npad);
    c->bk.pzmin = carve<uint32_t>(c, c->npad);
    c->bk.pzmax = carve<uint32_t>(c, c->npad);
    c->bk.rec = carve<uint4>(c, c->npad);
    c->bk.tsum = carve<uint32_t>(c, c->ntiles);
    c->bk.toff = carve<uint32_t>(c, c->ntiles);
    c->bk.tz = carve<float2>(c, c->ntiles);
    c->bk.vpix = carve<int>(c, V);
    c->bk.vslot = carve<uint32_t>(c, V);
    c->bk.sorted = carve<float4>(c, V);
    c->bk.bstat = carve<int4>(c, c->nassoc);
    c->bk.cellrec = carve<uint4>(c, 4 * (size_t)c->ntiles);
    c->acc.cnt = carve<uint32_t>(c, V);
    c->acc.sx = carve<long long>(c, V);
    c->acc.sy = carve<long long>(c, V);
    c->acc.sz = carve<long long>(c, V);
    c->assoc = carve<int32_t>(c, N);
    c->dstats = carve<DevStats>(c, 1);
    // ---- host-side tables, uploaded once ----
    std::vector<float> h(3 * V);
    for (size_t i = 0; i < V; ++i) { h[i] = model->rest_xyz[3 * i]; h[V + i] = model->rest_xyz[3 * i + 1]; h[2 * V + i] = model->rest_xyz[3 * i + 2]; }
    std::vector<float4> hw(V);
    std::vector<uint32_t> hl(V);
    for (size_t i = 0; i < V; ++i) {
        float ws[4] = {0, 0, 0, 0};
        uint32_t packed = 0xFFFFFFFFu;
        for (int k = 0; k < c->K; ++k) {
            int l = model->skin_link[i * c->K + k];
            if (l < 0) continue;
            ws[k] = model->skin_w[i * c->K + k];
            packed &= ~(0xFFu << (8 * k));
            packed |= (uint32_t)l << (8 * k);
        }
        hw[i] = make_float4(ws[0], ws[1], ws[2], ws[3]);
        hl[i] = packed;
    }
    std::vector<int> nbv;
    if (model->neighbors) nbv.assign(model->neighbors, model->neighbors + 4 * V);
    else nbv = nearest4(model->rest_xyz, c->V);
    std::vector<int4> hn(V);
    for (size_t i = 0; i < V; ++i) hn[i] = make_int4(nbv[4 * i], nbv[4 * i + 1], nbv[4 * i + 2], nbv[4 * i + 3]);
    std::vector<uint32_t> hoff(V + 1, 0);
    for (int64_t q = 0; q < 3 * (int64_t)c->F; ++q) hoff[model->faces[q] + 1]++;
    for (size_t i = 0; i < V; ++i) hoff[i + 1] += hoff[i];
    std::vector<int2> hfan(3 * (size_t)c->F);
    std::vector<uint32_t> fill(hoff.begin(), hoff.end() - 1);
    for (int f = 0; f < c->F; ++f) {
        int a = model->faces[3 * f], b = model->faces[3 * f + 1], d = model->faces[3 * f + 2];
        hfan[fill[a]++] = make_int2(b, d);
        hfan[fill[b]++] = make_int2(d, a);
        hfan[fill[d]++] = make_int2(a, b);
    }
    std::vector<uint32_t> hanc(4 * (size_t)c->L);
    for (int l = 0; l < c->L; ++l)
        for (int q = 0; q < 4; ++q) hanc[4 * l + q] = c->hjt.anc[l][q];
    auto up = [&](void* d, const void* s, size_t n) { return hipMemcpy(d, s, n, hipMemcpyHostToDevice) == hipSuccess; };
    bool ok = up(rest.x, h.data(), 4 * V) && up(rest.y, h.data() + V, 4 * V) && up(rest.z, h.data() + 2 * V, 4 * V) &&
              up(w4, hw.data(), 16 * V) && up(lk, hl.data(), 4 * V) && up(nb, hn.data(), 16 * V) &&
              up(fan_off, hoff.data(), 4 * (V + 1)) && (c->F == 0 || up(fan, hfan.data(), 8 * 3 * (size_t)c->F)) &&
              up(c->anc, hanc.data(), 4 * hanc.size()) && up(c->djt, &c->hjt, sizeof(JointTable)) &&
              up(c->theta, theta0, 8 * (size_t)c->P);
    if (!ok) { free_ctx(c); return fail(TRACK_E_DEVICE, "upload failed"); }
    c->dm = DevModel{c->P, c->L, c->V, c->F, rest.x, rest.y, rest.z, w4, lk, nb, fan_off, fan};
    float fmax = std::max(camera->fx, camera->fy);
    double ex = std::max((double)camera->cx + 0.5, (double)camera->width - 0.5 - camera->cx) / camera->fx;
    double ey = std::max((double)camera->cy + 0.5, (double)camera->height - 0.5 - camera->cy) / camera->fy;
    double rmax = std::sqrt(1.0 + ex * ex + ey * ey);
    c->dc = DevCam{c->W, c->H, tx, ty, camera->fx, camera->fy, camera->cx, camera->cy,
                   (float)((1.0 - 1e-4) / (fmax * rmax))};
    if (hipEventCreate(&c->f0) != hipSuccess || hipEventCreate(&c->f1) != hipSuccess) {
        free_ctx(c);
        return fail(TRACK_E_DEVICE, "event creation failed");
    }
    std::vector<float> z3(3 * V, 0.0f);
    const float* p0 = phi0 ? phi0 : z3.data();
    if ((rc = upload_soa(c, c->phi[0], p0)) || (rc = upload_soa(c, c->phi_prev, p0))) { free_ctx(c); return rc; }
    if (hipMemset(c->dstats, 0, sizeof(DevStats)) != hipSuccess) { free_ctx(c); return fail(TRACK_E_DEVICE, "memset"); }
    launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
    ensure_surface(c);
    if (hipStreamSynchronize(c->stream) != hipSuccess) { free_ctx(c); return fail(TRACK_E_DEVICE, "init kernels failed"); }
    *out = c;
    return TRACK_OK;
}

int track_set_params(track_ctx* c, const track_params* p) {
    if (!c) return fail(TRACK_E_INVALID, "ctx is NULL");
    return set_params(c, p);
}

int track_frame(track_ctx* c, const float* depth, int32_t on_device) {
    if (!c || !depth) return fail(TRACK_E_INVALID, "ctx/depth is NULL");
    const float* d = depth;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(c->depth_buf, depth, sizeof(float) * c->W * c->H, hipMemcpyHostToDevice, c->stream));
        d = c->depth_buf;
    }
    return run_frame(c, d, nullptr);
}

int track_frame_xyz(track_ctx* c, const float* xyz, int32_t on_device) {
    if (!c || !xyz) return fail(TRACK_E_INVALID, "ctx/xyz is NULL");
    const float* d = xyz;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(c->xyz_buf, xyz, sizeof(float) * 3 * c->W * c->H, hipMemcpyHostToDevice, c->stream));
        d = c->xyz_buf;
    }
    return run_frame(c, nullptr, d);
}

int track_state(const track_ctx* cc, double* theta, float* phi, float* verts, track_frame_stats* stats) {
    track_ctx* c = const_cast<track_ctx*>(cc);
    if (!c) return fail(TRACK_E_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (theta) HIP_TRY(hipMemcpy(theta, c->theta, sizeof(double) * c->P, hipMemcpyDeviceToHost));
    int rc;
    if (phi && (rc = download_soa(c, c->phi[c->phi_cur], phi))) return rc;
    if (verts) {
        ensure_surface(c);
        HIP_TRY(hipStreamSynchronize(c->stream));
        if ((rc = download_v4(c, c->verts[c->v_cur], verts))) return rc;
    }
    if (stats) *stats = c->last;
    return TRACK_OK;
}

int track_reset(track_ctx* c, const double* theta, const float* phi) {
    if (!c || !theta) return fail(TRACK_E_INVALID, "ctx/theta is NULL");
    for (int k = 0; k < c->P; ++k)
        if (!std::isfinite(theta[k])) return fail(TRACK_E_INVALID, "theta not finite");
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->theta, theta, sizeof(double) * c->P, hipMemcpyHostToDevice));
    std::vector<float> z3(3 * (size_t)c->V, 0.0f);
    const float* p0 = phi ? phi : z3.data();
    int rc;
    if ((rc = upload_soa(c, c->phi[c->phi_cur], p0)) || (rc = upload_soa(c, c->phi_prev, p0))) return rc;
    launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
    c->surface_valid = false;
    ensure_surface(c);
    HIP_TRY(hipStreamSynchronize(c->stream));
    return TRACK_OK;
}

void track_destroy(track_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

int track_kernel_timing(track_ctx* c, int32_t k, int32_t enable) {
    if (!c || k < 0 || k >= TRACK_K_COUNT_) return fail(TRACK_E_INVALID, "bad kernel id");
    HIP_TRY(hipStreamSynchronize(c->stream));
    timed_collect(c);
    c->timers[k].on = enable != 0;
    c->timers[k].launches = 0;
    c->timers[k].total_ms = 0.0;
    return TRACK_OK;
}

int track_kernel_time(track_ctx* c, int32_t k, int64_t* launches, double* total_ms) {
    if (!c || k < 0 || k >= TRACK_K_COUNT_) return fail(TRACK_E_INVALID, "bad kernel id");
    HIP_TRY(hipStreamSynchronize(c->stream));
    timed_collect(c);
    if (launches) *launches = c->timers[k].launches;
    if (total_ms) *total_ms = c->timers[k].total_ms;
    return TRACK_OK;
}

// ---- per-pass access -------------------------------------------------------
int track_dbg_set(track_ctx* c, int32_t buf, const void* host, size_t bytes) {
    if (!c || !host) return fail(TRACK_E_INVALID, "ctx/host is NULL");
    const size_t V = c->V, N = (size_t)c->W * c->H;
    HIP_TRY(hipStreamSynchronize(c->stream));
    switch (buf) {
        case TRACK_BUF_THETA:
            if (bytes != 8 * (size_t)c->P) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(c->theta, host, bytes, hipMemcpyHostToDevice));
            launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
            break;
        case TRACK_BUF_PHI:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return upload_soa(c, c->phi[c->phi_cur], (const float*)host);
        case TRACK_BUF_PHI_PREV:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return upload_soa(c, c->phi_prev, (const float*)host);
        case TRACK_BUF_VERTS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            c->surface_valid = true;
            return upload_v4(c, c->verts[c->v_cur], (const float*)host);
        case TRACK_BUF_NORMALS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return upload_soa(c, c->normals, (const float*)host);
        case TRACK_BUF_DEPTH:
            if (bytes != 4 * N) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(c->depth_buf, host, bytes, hipMemcpyHostToDevice));
            c->input_mode = 0;
            break;
        case TRACK_BUF_XYZ:
            if (bytes != 12 * N) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(c->xyz_buf, host, bytes, hipMemcpyHostToDevice));
            c->input_mode = 1;
            break;
        case TRACK_BUF_COUNT: {
            if (bytes != 4 * V) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(c->acc.cnt, host, bytes, hipMemcpyHostToDevice));
            break;
        }
        case TRACK_BUF_DELTA: {
            // stored as fixed-point sums: count * delta * 2^32 (set COUNT first)
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            std::vector<uint32_t> cnt(V);
            HIP_TRY(hipMemcpy(cnt.data(), c->acc.cnt, 4 * V, hipMemcpyDeviceToHost));
            const float* d = (const float*)host;
            std::vector<long long> s[3];
            for (int q = 0; q < 3; ++q) s[q].resize(V);
            for (size_t i = 0; i < V; ++i)
                for (int q = 0; q < 3; ++q) s[q][i] = std::llround((double)d[3 * i + q] * cnt[i] * kFix);
            HIP_TRY(hipMemcpy(c->acc.sx, s[0].data(), 8 * V, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(c->acc.sy, s[1].data(), 8 * V, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(c->acc.sz, s[2].data(), 8 * V, hipMemcpyHostToDevice));
            break;
        }
        default:
            return fail(TRACK_E_INVALID, "buffer cannot be set");
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return TRACK_OK;
}

int track_dbg_get(const track_ctx* cc, int32_t buf, void* host, size_t bytes) {
    track_ctx* c = const_cast<track_ctx*>(cc);
    if (!c || !host) return fail(TRACK_E_INVALID, "ctx/host is NULL");
    const size_t V = c->V, N = (size_t)c->W * c->H;
    HIP_TRY(hipStreamSynchronize(c->stream));
    switch (buf) {
        case TRACK_BUF_THETA:
            if (bytes != 8 * (size_t)c->P) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, c->theta, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_STEP:
            if (bytes != 8 * (size_t)c->P) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, c->step, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_PHI:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_soa(c, c->phi[c->phi_cur], (float*)host);
        case TRACK_BUF_PHI_PREV:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_soa(c, c->phi_prev, (float*)host);
        case TRACK_BUF_VERTS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_v4(c, c->verts[c->v_cur], (float*)host);
        case TRACK_BUF_VERTS_NEW:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_v4(c, c->verts[c->v_cur], (float*)host);
        case TRACK_BUF_NORMALS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_soa(c, c->normals, (float*)host);
        case TRACK_BUF_ASSOC:
            if (bytes != 4 * N) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, c->assoc, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_COUNT:
            if (bytes != 4 * V) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, c->acc.cnt, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_DELTA: {
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            std::vector<uint32_t> cnt(V);
            std::vector<long long> s[3];
            HIP_TRY(hipMemcpy(cnt.data(), c->acc.cnt, 4 * V, hipMemcpyDeviceToHost));
            long long* src[3] = {c->acc.sx, c->acc.sy, c->acc.sz};
            for (int q = 0; q < 3; ++q) {
                s[q].resize(V);
                HIP_TRY(hipMemcpy(s[q].data(), src[q], 8 * V, hipMemcpyDeviceToHost));
            }
            float* d = (float*)host;
            for (size_t i = 0; i < V; ++i)
                for (int q = 0; q < 3; ++q)
                    d[3 * i + q] = cnt[i] ? (float)((double)s[q][i] / ((double)cnt[i] * kFix)) : 0.0f;
            return TRACK_OK;
        }
        case TRACK_BUF_GRAM: {
            const size_t n1 = (size_t)c->P + 1;
            if (bytes != 8 * n1 * n1) return fail(TRACK_E_INVALID, "size");
            std::vector<double> g((size_t)c->PP * c->PP);
            HIP_TRY(hipMemcpy(g.data(), c->gram, 8 * g.size(), hipMemcpyDeviceToHost));
            double* d = (double*)host;
            for (size_t i = 0; i < n1; ++i)
                for (size_t j = 0; j < n1; ++j) d[i * n1 + j] = g[i * c->PP + j];
            return TRACK_OK;
        }
        default:
            return fail(TRACK_E_INVALID, "buffer cannot be read");
    }
}

int track_dbg_run(track_ctx* c, int32_t pass) {
    if (!c) return fail(TRACK_E_INVALID, "ctx is NULL");
    const float* depth = c->input_mode == 0 ? c->depth_buf : nullptr;
    const float* xyz = c->input_mode == 1 ? c->xyz_buf : nullptr;
    switch (pass) {
        case TRACK_PASS_SKIN:
            launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
            c->surface_valid = false;
            ensure_surface(c);
            break;
        case TRACK_PASS_NORMALS:
            launch_normals(c->stream, c->dm, c->verts[c->v_cur], c->normals);
            break;
        case TRACK_PASS_ASSOCIATE:
            pass_associate(c, depth, xyz);
            break;
        case TRACK_PASS_NORMAL_EQ:
            launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
            pass_normal_eq(c);
            break;
        case TRACK_PASS_POSE_STEP:
            HIP_TRY(hipMemsetAsync(&c->dstats->status, 0, sizeof(int), c->stream));
            pass_pose_step(c, 0);
            break;
        case TRACK_PASS_SHAPE:
            launch_fk(c->stream, c->djt, c->theta, c->dq, c->xi);
            pass_shape(c, true);
            break;
        default:
            return fail(TRACK_E_INVALID, "unknown pass");
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (pass == TRACK_PASS_POSE_STEP) {
        int st = 0;
        HIP_TRY(hipMemcpy(&st, &c->dstats->status, sizeof(int), hipMemcpyDeviceToHost));
        if (st == TRACK_E_NOT_PD) return fail(TRACK_E_NOT_PD, "pose system not positive definite");
    }
    return TRACK_OK;
}

}  // extern "C"
