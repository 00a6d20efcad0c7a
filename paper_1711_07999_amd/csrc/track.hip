// Host runtime and C ABI of libtrack: model preparation, device memory, the
// per-frame iteration schedule (Section 4), the batched serving loop and
// per-pass access.
//
// Every kernel runs over a batch of tracking streams described by a device
// slot table (common.h).  A context (track_ctx) is a batch of one whose
// frames are captured once as HIP graphs and replayed; a server
// (track_server) batches every resident stream into the same launches, one
// Gauss-Newton iteration per step, so streams join and leave at iteration
// boundaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <bitset>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/track.h"
#include "common.h"

using namespace trk;

// Working memory of allocation-free frames (track_frame_noalloc): one block
// per GPU, held until the process ends, shared by every such call on that
// GPU.  Host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (scratch_base).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

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

int validate_model(const track_model* m, const track_camera* cam) {
    if (!m || !cam) return fail(TRACK_E_INVALID, "model/camera is NULL");
    if (m->n_joints < 1 || m->n_joints > TRACK_MAX_JOINTS) return fail(TRACK_E_INVALID, "n_joints out of range");
    if (m->n_links < 1 || m->n_links > TRACK_MAX_LINKS) return fail(TRACK_E_INVALID, "n_links out of range");
    if (m->n_verts < 1) return fail(TRACK_E_INVALID, "n_verts must be >= 1");
    if (m->n_faces < 0) return fail(TRACK_E_INVALID, "n_faces must be >= 0");
    if (m->max_infl < 1 || m->max_infl > TRACK_MAX_INFL) return fail(TRACK_E_INVALID, "max_infl out of range");
    if (m->blend != TRACK_BLEND_DQ && m->blend != TRACK_BLEND_LINEAR) return fail(TRACK_E_INVALID, "unknown blend");
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
    if (!(m->scale > 0.0f) || !std::isfinite(m->scale)) return fail(TRACK_E_INVALID, "model scale must be > 0");
    if (cam->width < 1 || cam->height < 1 || cam->width > 4096 || cam->height > 4096)
        return fail(TRACK_E_INVALID, "image size out of range");
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !std::isfinite(cam->fx) || !std::isfinite(cam->fy) ||
        !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
        return fail(TRACK_E_INVALID, "bad camera intrinsics");
    return TRACK_OK;
}

int validate_params(const track_params* p, int P) {
    if (!p) return fail(TRACK_E_INVALID, "params is NULL");
    if (!(p->tau > 0.0f) || !std::isfinite(p->tau)) return fail(TRACK_E_INVALID, "tau must be > 0");
    if (p->n_iters < 1 || p->n_iters > 256) return fail(TRACK_E_INVALID, "n_iters must be in 1..256");
    if (!p->do_pose || !p->do_shape) return fail(TRACK_E_INVALID, "do_pose/do_shape are required");
    if (p->gram_mode != TRACK_GRAM_FP32 && p->gram_mode != TRACK_GRAM_BF16X3 && p->gram_mode != TRACK_GRAM_BF16X6)
        return fail(TRACK_E_INVALID, "unknown gram_mode");
    const float lam[6] = {p->lambda_k, p->lambda_s, p->lambda_phi, p->lambda_nbr, p->lambda_t, p->lambda_w};
    for (float l : lam)
        if (!(l >= 0.0f) || !std::isfinite(l)) return fail(TRACK_E_INVALID, "weights must be finite and >= 0");
    (void)P;
    return TRACK_OK;
}

// The template resized by its uniform scale s about c, the translation of
// joint 0's offset (Section 5.4 sizes the template to the subject this way):
// rest vertices x -> c + s (x - c), offsets of joints with a parent t -> s t,
// of other root joints t -> c + s (t - c); arithmetic in float64, rounded
// once.  Arrays the scale leaves alone stay the caller's.
struct ScaledModel {
    track_model m{};
    std::vector<float> rest, offset;
    const track_model* apply(const track_model* in) {
        if (in->scale == 1.0f) return in;
        m = *in;
        const double sc = in->scale;
        const double c[3] = {in->joint_offset[4], in->joint_offset[5], in->joint_offset[6]};
        rest.resize(3 * (size_t)in->n_verts);
        for (size_t q = 0; q < rest.size(); ++q) rest[q] = (float)(c[q % 3] + sc * ((double)in->rest_xyz[q] - c[q % 3]));
        offset.assign(in->joint_offset, in->joint_offset + 7 * (size_t)in->n_joints);
        for (int j = 0; j < in->n_joints; ++j)
            for (int d = 0; d < 3; ++d) {
                const double t = in->joint_offset[7 * j + 4 + d];
                offset[7 * j + 4 + d] = (float)(in->joint_parent[j] >= 0 ? sc * t : c[d] + sc * (t - c[d]));
            }
        m.rest_xyz = rest.data();
        m.joint_offset = offset.data();
        m.scale = 1.0f;
        return &m;
    }
};

// Device memory of a context or stream: the caller's provider, else hipMalloc.
void* dev_alloc(const track_allocator& a, size_t bytes) {
    void* p = nullptr;
    if (a.alloc) {
        p = a.alloc(bytes, a.user);
        if (p && (reinterpret_cast<uintptr_t>(p) & 255u)) {  // the layout assumes 256-byte alignment
            if (a.free) a.free(p, a.user);
            p = nullptr;
        }
        return p;
    }
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dev_free(const track_allocator& a, void* p) {
    if (!p) return;
    if (a.alloc) {
        if (a.free) a.free(p, a.user);
    } else {
        (void)hipFree(p);
    }
}

// ---------------------------------------------------------------------------
// The iteration schedule shared by the streams of a batch.
// ---------------------------------------------------------------------------
struct Schedule {
    int n_iters = 1;
    std::vector<uint8_t> do_pose, do_shape;
    int gram_mode = 0, pose_fp64 = 0, shape_fp64 = 0;
    int first_pose = -1, last_pose = -1;

    void set(const track_params* p) {
        n_iters = p->n_iters;
        do_pose.assign(p->do_pose, p->do_pose + n_iters);
        do_shape.assign(p->do_shape, p->do_shape + n_iters);
        gram_mode = p->gram_mode;
        pose_fp64 = p->pose_solve_fp64 ? 1 : 0;
        shape_fp64 = p->shape_solve_fp64 ? 1 : 0;
        first_pose = last_pose = -1;
        for (int t = 0; t < n_iters; ++t)
            if (do_pose[t]) { if (first_pose < 0) first_pose = t; last_pose = t; }
    }
};

// ---------------------------------------------------------------------------
// One tracking stream's device state: model tables, per-frame buffers and
// the host's record of which vertex and offset buffers are current.
// ---------------------------------------------------------------------------
struct Stream {
    int P = 0, L = 0, V = 0, F = 0, K = 0, PP = 0, W = 0, H = 0, ntiles = 0, negrid = 0;
    int blend = TRACK_BLEND_DQ;
    JointTable hjt{};
    JointTable* djt = nullptr;
    TreePlan hplan{};             // tree form of the pose solve (pointers: device addresses once carved)
    std::vector<uint32_t> hblob;
    std::vector<int> hgfmap;
    std::vector<double> prior_S;  // S_k: share of vertices each joint moves
    void* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    track_allocator alloc{};       // where the arena came from (all null: hipMalloc)
    Slot slot{};                   // device pointers and constants of this stream
    float *depth_buf = nullptr, *xyz_buf = nullptr;
    int v_cur = 0, phi_cur = 0, phi_prev = 0;
    int bpar = 0;                  // bucket counters the next count fills (the other parity holds the last ones)
    bool surface_valid = false, refresh_pose = true;
    bool dirty = true;             // buckets / accumulators not known to be clear
    bool buckets_ready = false;    // the other bucket parity holds the last association's counts
    int input_mode = 0;            // per-pass interface: 0 depth, 1 xyz
};

template <class T>
T* carve(Stream* s, size_t n) {
    size_t bytes = (n * sizeof(T) + 255) & ~size_t(255);
    T* p = s->arena ? reinterpret_cast<T*>(static_cast<char*>(s->arena) + s->arena_used) : nullptr;
    s->arena_used += bytes;
    return p;
}

void build_tree_plan(Stream* c, const track_model* m);

void build_joint_table(Stream* c, const track_model* m) {
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
    // pointer-jumping rounds of forward kinematics: ceil(log2(chain length))
    int longest = 1;
    for (int j = 0; j < t.P; ++j) {
        int d = 1;
        for (int k = t.parent[j]; k >= 0; k = t.parent[k]) ++d;
        longest = std::max(longest, d);
    }
    t.rounds = 0;
    while ((1 << t.rounds) < longest) ++t.rounds;
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
    build_tree_plan(c, m);
}

// Tree form of the pose solve.  A_kj can be non-zero only if some vertex
// has weight on links whose chains (Section 3.1) hold both k and j; with the
// joints eliminated children first (parent indices are smaller) the factor
// keeps to the fill of that pattern, computed here symbolically, and its
// elimination tree follows the limbs.  Chains of the elimination tree whose
// nodes have one child each become supernodes.  Fronts wider than
// kFrontRows - 1 rows, or storage beyond what the kernel's LDS allows, leave
// the model to the dense form.
void build_tree_plan(Stream* c, const track_model* m) {
    TreePlan& t = c->hplan;
    std::memset(&t, 0, sizeof(t));
    c->hblob.clear();
    c->hgfmap.clear();
    const char* env = std::getenv("TRACK_DENSE_SOLVE");
    if (env && env[0] == '1') return;
    const int P = c->P;
    const JointTable& jt = c->hjt;
    // distinct chain unions over the vertices
    std::set<std::array<uint32_t, 4>> masks;
    for (int i = 0; i < m->n_verts; ++i) {
        std::array<uint32_t, 4> mk{0, 0, 0, 0};
        for (int k = 0; k < m->max_infl; ++k) {
            const int l = m->skin_link[i * m->max_infl + k];
            if (l >= 0 && m->skin_w[i * m->max_infl + k] > 0.0f)
                for (int q = 0; q < 4; ++q) mk[q] |= jt.anc[l][q];
        }
        masks.insert(mk);
    }
    // column structure in elimination positions: joint j sits at P - 1 - j
    std::vector<std::bitset<kMaxJoints + 1>> st(P);
    for (const auto& mk : masks) {
        std::vector<int> js;
        for (int j = 0; j < P; ++j)
            if ((mk[j >> 5] >> (j & 31)) & 1u) js.push_back(P - 1 - j);
        for (int a : js)
            for (int b : js)
                if (a > b) st[b].set(a);
    }
    std::vector<int> epar(P, -1), nchild(P, 0);
    for (int p = 0; p < P; ++p) {
        if (st[p].none()) continue;
        int q = p + 1;
        while (!st[p].test(q)) ++q;
        epar[p] = q;
        nchild[q] += 1;
        auto rest = st[p];
        rest.reset(q);
        st[q] |= rest;
    }
    // supernodes: runs p, p + 1, ... where p + 1 is the only child's parent
    std::vector<int> sfirst, slast, snof(P);
    for (int p = 0; p < P;) {
        const int a = p;
        if ((int)st[p].count() + 2 > kFrontRows) return;
        while (p + 1 < P && epar[p] == p + 1 && nchild[p + 1] == 1 &&
               (p + 2 - a) + (int)st[p + 1].count() + 1 <= kFrontRows)
            ++p;
        for (int q = a; q <= p; ++q) snof[q] = (int)sfirst.size();
        sfirst.push_back(a);
        slast.push_back(p);
        ++p;
    }
    const int nsn = (int)sfirst.size();
    std::vector<int> spar(nsn, -1), lev(nsn, 0);
    std::vector<std::vector<int>> rows(nsn);   // elimination positions, increasing
    for (int s = 0; s < nsn; ++s) {
        for (int q = sfirst[s]; q <= slast[s]; ++q) rows[s].push_back(q);
        for (int q = slast[s] + 1; q < P; ++q)
            if (st[slast[s]].test(q)) rows[s].push_back(q);
        if (epar[slast[s]] >= 0) spar[s] = snof[epar[slast[s]]];
    }
    for (int s = 0; s < nsn; ++s)   // children come before their parents
        if (spar[s] >= 0) lev[spar[s]] = std::max(lev[spar[s]], lev[s] + 1);
    int nlev = 0;
    for (int s = 0; s < nsn; ++s) nlev = std::max(nlev, lev[s] + 1);
    // fronts
    struct Fr { int off, np, f, fw; };
    std::vector<Fr> fr(nsn);
    std::vector<std::vector<int>> joint(nsn);   // front row -> joint
    int elems = 0;
    for (int s = 0; s < nsn; ++s) {
        Fr& F = fr[s];
        F.np = slast[s] - sfirst[s] + 1;
        F.f = (int)rows[s].size();
        F.fw = F.f + 1 <= 8 ? 8 : F.f + 1 <= 16 ? 16 : F.f + 1 <= 24 ? 24 : 32;   // the kernel's register widths
        F.off = elems;
        elems += (F.f + 1) * F.fw;
        for (int r = 0; r < F.f; ++r) joint[s].push_back(P - 1 - rows[s][r]);
    }
    if (elems >= (1 << 15)) return;
    // assembly rounds of each parent: its children's update blocks (lower
    // triangle and right-hand-side row), children in index order, each parent
    // entry at most once per round
    std::vector<std::vector<uint32_t>> rounds(nsn);
    for (int s = 0; s < nsn; ++s) {
        std::vector<std::vector<uint32_t>> rr;
        std::vector<int> last_round((size_t)(fr[s].f + 1) * fr[s].fw, -1);
        for (int ch = 0; ch < nsn; ++ch) {
            if (spar[ch] != s) continue;
            const Fr& C = fr[ch];
            const int nU = C.f - C.np;
            std::vector<int> pos(nU);
            for (int u = 0; u < nU; ++u)
                pos[u] = (int)(std::lower_bound(rows[s].begin(), rows[s].end(), rows[ch][C.np + u]) - rows[s].begin());
            for (int i = 0; i <= nU; ++i)
                for (int j = 0; j < nU && j <= i; ++j) {
                    const int prow = i < nU ? pos[i] : fr[s].f;
                    const int dst = prow * fr[s].fw + pos[j];
                    const int src = C.off + (C.np + i) * C.fw + C.np + j;
                    int r = last_round[dst] + 1;
                    while (r < (int)rr.size() && rr[r].size() >= 64) ++r;
                    if (r == (int)rr.size()) rr.emplace_back();
                    rr[r].push_back((uint32_t)src | ((uint32_t)(fr[s].off + dst) << 16));
                    last_round[dst] = r;
                }
        }
        for (auto& q : rr) {
            q.resize(64, 0xFFFF0000u);
            rounds[s].insert(rounds[s].end(), q.begin(), q.end());
        }
    }
    // per level, longest processing time first over the waves (cost: pivots x
    // width); a front goes to the least loaded SIMD (waves w and w + 4 of the
    // workgroup share one), then to its less loaded wave, so the longest
    // fronts do not share an issue port
    std::vector<int> wstart((size_t)nlev * kSolveWaves + 1), sched;
    for (int l = 0; l < nlev; ++l) {
        std::vector<int> ids;
        for (int s = 0; s < nsn; ++s)
            if (lev[s] == l) ids.push_back(s);
        auto cost = [&](int s) { return (int64_t)fr[s].np * fr[s].fw + (int64_t)rounds[s].size(); };
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return cost(a) > cost(b); });
        std::vector<std::vector<int>> per(kSolveWaves);
        std::vector<int64_t> load(kSolveWaves, 0);
        auto simd_load = [&](int w) {
            int64_t t = 0;
            for (int v = w % 4; v < kSolveWaves; v += 4) t += load[v];
            return t;
        };
        for (int s : ids) {
            int w = 0;
            for (int v = 1; v < kSolveWaves; ++v) {
                const int64_t lv = simd_load(v), lw = simd_load(w);
                if (lv < lw || (lv == lw && load[v] < load[w])) w = v;
            }
            per[w].push_back(s);
            load[w] += cost(s);
        }
        for (int w = 0; w < kSolveWaves; ++w) {
            wstart[l * kSolveWaves + w] = (int)sched.size();
            for (int s : per[w]) sched.push_back(s);
        }
    }
    wstart[(size_t)nlev * kSolveWaves] = (int)sched.size();
    // the blob
    std::vector<uint32_t>& B = c->hblob;
    B.assign(wstart.begin(), wstart.end());
    t.o_sched = (int)B.size();
    B.insert(B.end(), sched.begin(), sched.end());
    t.o_front = (int)B.size();
    B.resize(B.size() + (size_t)kFrontWords * nsn, 0u);
    std::vector<int> amap0(nsn);
    for (int s = 0; s < nsn; ++s) {
        amap0[s] = (int)B.size();
        B.insert(B.end(), rounds[s].begin(), rounds[s].end());
    }
    std::vector<int> row0(nsn);
    std::vector<unsigned char> bytes;
    const int rbase = (int)B.size() * 4;
    for (int s = 0; s < nsn; ++s) {
        row0[s] = rbase + (int)bytes.size();
        for (int r = 0; r < fr[s].f; ++r) bytes.push_back((unsigned char)joint[s][r]);
    }
    bytes.resize((bytes.size() + 3) & ~size_t(3), 0);
    for (size_t q = 0; q < bytes.size(); q += 4)
        B.push_back((uint32_t)bytes[q] | ((uint32_t)bytes[q + 1] << 8) | ((uint32_t)bytes[q + 2] << 16) |
                    ((uint32_t)bytes[q + 3] << 24));
    for (int s = 0; s < nsn; ++s) {
        uint32_t* w = &B[(size_t)t.o_front + (size_t)kFrontWords * s];
        w[0] = fr[s].off; w[1] = fr[s].np; w[2] = fr[s].f; w[3] = fr[s].fw;
        w[4] = amap0[s]; w[5] = (uint32_t)(rounds[s].size() / 64); w[6] = row0[s]; w[7] = 0;
    }
    // where the Gram reduction puts each element: the lower triangle of
    // each front's pivot columns and the right-hand side of its pivots
    // (column P).  All sit at or above the Gram diagonal: a front's later
    // rows hold smaller joint indices.
    c->hgfmap.assign((size_t)c->PP * c->PP, -1);
    for (int s = 0; s < nsn; ++s) {
        const Fr& F = fr[s];
        for (int i = 0; i <= F.f; ++i)
            for (int j = 0; j < F.np; ++j) {
                if (i < F.f && j > i) continue;
                const int gi = i < F.f ? joint[s][i] : joint[s][j];
                const int gj = i < F.f ? joint[s][j] : P;
                c->hgfmap[(size_t)gi * c->PP + gj] = F.off + i * F.fw + j;
            }
    }
    t.nsn = nsn;
    t.nlev = nlev;
    t.elems = elems;
    t.nwords = (int)B.size();
    t.ok = tree_solve_fits(elems, t.nwords) ? 1 : 0;
}

// per-stream constants: association cutoff, weights, prior and active mask
int stream_set_params(Stream* c, const track_params* p) {
    Slot& S = c->slot;
    S.tau = p->tau;
    S.lambda_k = p->lambda_k;
    S.lphi = p->lambda_phi;
    S.lnbr = p->lambda_nbr;
    S.lt = p->lambda_t;
    S.lw = p->lambda_w;
    for (int k = 0; k < c->P; ++k) {
        double w = (double)p->lambda_s * c->prior_S[k];
        c->hjt.prior[k] = w * w;
        c->hjt.active[k] = p->active ? (p->active[k] ? 1 : 0) : 1;
    }
    if (c->djt) HIP_TRY(hipMemcpy(c->djt, &c->hjt, sizeof(JointTable), hipMemcpyHostToDevice));
    return TRACK_OK;
}

// The association's tile order.  Workgroups are dealt to the XCDs in turn
// (workgroup b runs on XCD b % 8), so entry k of the order runs on XCD k % 8.
// Each XCD takes whole blocks of 4x4 tiles (block (bx, by) on XCD
// (bx + 3 by) % 8: neighbouring blocks on different XCDs, the subject spread
// over all of them), so that a tile's neighbours -- whose cells its search
// reads -- mostly share its XCD's L2; within an XCD, tiles nearest the
// principal point first (where the subject and the longest searches usually
// are; ties: index).  Lists of unequal length leave -1 entries.
std::vector<int> tile_order(int tx, int ty, double cx, double cy) {
    std::vector<std::vector<int>> lists(kXcds);
    for (int t = 0; t < tx * ty; ++t) {
        const int bx = (t % tx) / 4, by = (t / tx) / 4;
        lists[(bx + 3 * by) % kXcds].push_back(t);
    }
    size_t len = 0;
    for (auto& l : lists) {
        std::stable_sort(l.begin(), l.end(), [&](int a, int b) {
            auto d = [&](int u) {
                const double dx = (u % tx) * 8 + 3.5 - cx, dy = (u / tx) * 8 + 3.5 - cy;
                return dx * dx + dy * dy;
            };
            return d(a) < d(b);
        });
        len = std::max(len, l.size());
    }
    std::vector<int> order(kXcds * len, -1);
    for (int x = 0; x < kXcds; ++x)
        for (size_t k = 0; k < lists[x].size(); ++k) order[kXcds * k + x] = lists[x][k];
    return order;
}

// Lay out the stream's device memory.  Without an arena only the size is
// accumulated (admission control uses it).
void stream_layout(Stream* c) {
    const size_t V = c->V, N = (size_t)c->W * c->H;
    c->arena_used = 0;
    Slot& S = c->slot;
    c->djt = carve<JointTable>(c, 1);
    S.theta = carve<double>(c, c->P);
    S.theta_backup = carve<double>(c, c->P);
    S.step = carve<double>(c, c->P);
    S.gram = carve<double>(c, (size_t)c->PP * c->PP);
    S.dq = carve<float>(c, 8 * c->L);
    S.xi = carve<float>(c, 8 * c->P);
    uint32_t* anc = carve<uint32_t>(c, 4 * c->L);
    S.anc = anc;
    S.partials = carve<float>(c, (size_t)c->negrid * c->PP * c->PP);
    c->hplan.blob = carve<uint32_t>(c, (size_t)std::max(4, (c->hplan.nwords + 3) / 4 * 4));
    {
        TreeRef& tr = S.tree;
        const TreePlan& t = c->hplan;
        tr.blob = t.blob;
        tr.fimg = carve<double>(c, (size_t)std::max(2, t.elems));
        int* gfmap = carve<int>(c, (size_t)c->PP * c->PP);
        tr.gfmap = t.ok ? gfmap : nullptr;
        tr.nwords = t.nwords; tr.nlev = t.nlev; tr.elems = t.elems;
        tr.o_sched = t.o_sched; tr.o_front = t.o_front;
    }
    c->depth_buf = carve<float>(c, N);
    c->xyz_buf = carve<float>(c, 3 * N);
    auto v3 = [&]() { Vec3Buf b; b.x = carve<float>(c, V); b.y = carve<float>(c, V); b.z = carve<float>(c, V); return b; };
    Vec3Buf rest = v3();
    for (int q = 0; q < 3; ++q) S.phi[q] = v3();
    S.verts[0] = carve<float4>(c, V);
    S.verts[1] = carve<float4>(c, V);
    S.normals = v3();
    S.m.rx = rest.x; S.m.ry = rest.y; S.m.rz = rest.z;
    S.m.w = carve<float4>(c, V);
    S.m.links = carve<uint32_t>(c, V);
    S.m.nbr = carve<int4>(c, V);
    S.m.fan_off = carve<uint32_t>(c, V + 1);
    S.m.fan = carve<int2>(c, 3 * (size_t)c->F);
    S.m.fan8 = carve<int2>(c, (size_t)kFanInline * V);
    Buckets& b = S.b;
    for (int q = 0; q < 2; ++q) {
        b.cells[q] = carve<uint4>(c, 4 * (size_t)c->ntiles + 1);
        b.tsum[q] = carve<uint32_t>(c, c->ntiles);
    }
    b.ovfn = carve<uint32_t>(c, 2);
    b.scnt = carve<uint32_t>(c, 2 * kXcds);
    b.tlist = carve<int>(c, kXcds * (size_t)screen_queue(c->ntiles));
    b.ncap = bucket_capacity(c->V, c->ntiles);
    b.cellv = carve<float4>(c, (size_t)b.ncap + V);
    b.ntorder = (int)tile_order((c->W + 7) / 8, (c->H + 7) / 8, 0.0, 0.0).size();
    b.torder = carve<int>(c, b.ntorder);
    b.capx = screen_queue(c->ntiles);
    b.bstat = carve<int4>(c, c->ntiles);
    S.a.cnt = carve<uint32_t>(c, V);
    S.a.sx = carve<long long>(c, V);
    S.a.sy = carve<long long>(c, V);
    S.a.sz = carve<long long>(c, V);
    S.assoc = carve<int32_t>(c, N);
    S.st = carve<DevStats>(c, 1);
}

// device bytes of a stream (arena plus joint table)
size_t stream_bytes(const track_model* m, const track_camera* cam) {
    Stream s;
    s.P = m->n_joints; s.L = m->n_links; s.V = m->n_verts; s.F = m->n_faces;
    s.PP = ((s.P + 1) + 15) / 16 * 16;
    s.W = cam->width; s.H = cam->height;
    s.ntiles = ((s.W + 7) / 8) * ((s.H + 7) / 8);
    s.negrid = ne_grid(s.V);
    stream_layout(&s);
    return s.arena_used;
}

// The buffers of a frame whose contents mean nothing outside it (Gram
// matrices, the solve's front image, bucket index, per-vertex sums,
// matches, a staging copy of a host depth image), laid out from `base` into
// the slot (base null: sizes only).  Returns the bytes used.
size_t frame_scratch_layout(const Stream* c, char* base, Slot& S, float** depth_stage) {
    size_t used = 0;
    auto take = [&](size_t n, size_t elem) -> void* {
        void* p = base ? base + used : nullptr;
        used += (n * elem + 255) & ~size_t(255);
        return p;
    };
    const size_t V = c->V, N = (size_t)c->W * c->H;
    S.gram = static_cast<double*>(take((size_t)c->PP * c->PP, sizeof(double)));
    S.partials = static_cast<float*>(take((size_t)c->negrid * c->PP * c->PP, sizeof(float)));
    S.tree.fimg = static_cast<double*>(take((size_t)std::max(2, c->hplan.elems), sizeof(double)));
    Buckets& b = S.b;
    for (int q = 0; q < 2; ++q) {
        b.cells[q] = static_cast<uint4*>(take(4 * (size_t)c->ntiles + 1, sizeof(uint4)));
        b.tsum[q] = static_cast<uint32_t*>(take(c->ntiles, sizeof(uint32_t)));
    }
    b.ovfn = static_cast<uint32_t*>(take(2, 4));
    b.scnt = static_cast<uint32_t*>(take(2 * kXcds, 4));
    b.tlist = static_cast<int*>(take(kXcds * (size_t)b.capx, 4));
    b.ncap = bucket_capacity(c->V, c->ntiles);
    b.cellv = static_cast<float4*>(take((size_t)b.ncap + V, sizeof(float4)));
    b.bstat = static_cast<int4*>(take(c->ntiles, sizeof(int4)));
    S.a.cnt = static_cast<uint32_t*>(take(V, 4));
    S.a.sx = static_cast<long long*>(take(V, 8));
    S.a.sy = static_cast<long long*>(take(V, 8));
    S.a.sz = static_cast<long long*>(take(V, 8));
    S.assoc = static_cast<int32_t*>(take(N, 4));
    float* d = static_cast<float*>(take(N, 4));
    if (depth_stage) *depth_stage = d;
    return used;
}

// Address of `scratch` on the current device, looked up once per device.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;

int scratch_base(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(TRACK_E_DEVICE, std::string("scratch block address: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TRACK_OK;
}

int upload_soa(int V, Vec3Buf dst, const float* aos) {
    std::vector<float> t(3 * (size_t)V);
    for (int i = 0; i < V; ++i) { t[i] = aos[3 * i]; t[V + i] = aos[3 * i + 1]; t[2 * (size_t)V + i] = aos[3 * i + 2]; }
    HIP_TRY(hipMemcpy(dst.x, t.data(), sizeof(float) * V, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dst.y, t.data() + V, sizeof(float) * V, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dst.z, t.data() + 2 * (size_t)V, sizeof(float) * V, hipMemcpyHostToDevice));
    return TRACK_OK;
}

int download_soa(int V, Vec3Buf src, float* aos) {
    std::vector<float> t(3 * (size_t)V);
    HIP_TRY(hipMemcpy(t.data(), src.x, sizeof(float) * V, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t.data() + V, src.y, sizeof(float) * V, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t.data() + 2 * (size_t)V, src.z, sizeof(float) * V, hipMemcpyDeviceToHost));
    for (int i = 0; i < V; ++i) { aos[3 * i] = t[i]; aos[3 * i + 1] = t[V + i]; aos[3 * i + 2] = t[2 * (size_t)V + i]; }
    return TRACK_OK;
}

int upload_v4(int V, float4* dst, const float* aos) {
    std::vector<float4> t(V);
    for (int i = 0; i < V; ++i) t[i] = make_float4(aos[3 * i], aos[3 * i + 1], aos[3 * i + 2], 0.0f);
    HIP_TRY(hipMemcpy(dst, t.data(), sizeof(float4) * V, hipMemcpyHostToDevice));
    return TRACK_OK;
}

int download_v4(int V, const float4* src, float* aos) {
    std::vector<float4> t(V);
    HIP_TRY(hipMemcpy(t.data(), src, sizeof(float4) * V, hipMemcpyDeviceToHost));
    for (int i = 0; i < V; ++i) { aos[3 * i] = t[i].x; aos[3 * i + 1] = t[i].y; aos[3 * i + 2] = t[i].z; }
    return TRACK_OK;
}

void stream_free(Stream* c) {
    if (!c) return;
    dev_free(c->alloc, c->arena);
    c->arena = nullptr;
    c->djt = nullptr;
}

// Allocate and fill a stream; on failure nothing stays allocated.
int stream_create(Stream* c, const track_model* model, const track_camera* camera, const track_params* params,
                  const double* theta0, const float* phi0, const track_allocator* alloc) {
    c->P = model->n_joints; c->L = model->n_links; c->V = model->n_verts; c->F = model->n_faces;
    c->K = model->max_infl;
    c->blend = model->blend;
    c->PP = ((c->P + 1) + 15) / 16 * 16;
    c->W = camera->width; c->H = camera->height;
    const int tx = (c->W + 7) / 8, ty = (c->H + 7) / 8;
    c->ntiles = tx * ty;
    c->negrid = ne_grid(c->V);
    build_joint_table(c, model);
    stream_layout(c);  // size only
    c->arena_bytes = c->arena_used;
    c->alloc = alloc ? *alloc : track_allocator{};
    c->arena = dev_alloc(c->alloc, c->arena_bytes);
    if (!c->arena) return fail(TRACK_E_NOMEM, "device allocation failed");
    stream_layout(c);  // carve
    Slot& S = c->slot;
    S.jt = c->djt;
    S.PP = c->PP;
    S.negrid = c->negrid;
    const size_t V = c->V;
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
    // the first kFanInline fan entries of each vertex, slot-major so that a
    // thread's loads are independent and a wave's coalesced
    std::vector<int2> hfan8((size_t)kFanInline * V);
    for (size_t i = 0; i < V; ++i)
        for (int k = 0; k < kFanInline; ++k) {
            const uint32_t e = hoff[i] + (uint32_t)k;
            hfan8[(size_t)k * V + i] = e < hoff[i + 1] ? hfan[e] : make_int2((int)i, (int)i);
        }
    std::vector<uint32_t> hanc(4 * (size_t)c->L);
    for (int l = 0; l < c->L; ++l)
        for (int q = 0; q < 4; ++q) hanc[4 * l + q] = c->hjt.anc[l][q];
    auto up = [&](const void* d, const void* s, size_t n) {
        return hipMemcpy(const_cast<void*>(d), s, n, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up(S.m.rx, h.data(), 4 * V) && up(S.m.ry, h.data() + V, 4 * V) && up(S.m.rz, h.data() + 2 * V, 4 * V) &&
              up(S.m.w, hw.data(), 16 * V) && up(S.m.links, hl.data(), 4 * V) && up(S.m.nbr, hn.data(), 16 * V) &&
              up(S.m.fan_off, hoff.data(), 4 * (V + 1)) && (c->F == 0 || up(S.m.fan, hfan.data(), 8 * 3 * (size_t)c->F)) &&
              up(S.m.fan8, hfan8.data(), sizeof(int2) * hfan8.size()) &&
              up(S.anc, hanc.data(), 4 * hanc.size()) && up(S.theta, theta0, 8 * (size_t)c->P) &&
              (!S.tree.gfmap || up(S.tree.gfmap, c->hgfmap.data(), sizeof(int) * c->hgfmap.size())) &&
              (c->hblob.empty() || up(c->hplan.blob, c->hblob.data(), sizeof(uint32_t) * c->hblob.size())) &&
              (!S.tree.gfmap || hipMemset(S.tree.fimg, 0, sizeof(double) * c->hplan.elems) == hipSuccess) &&
              hipMemset(S.st, 0, sizeof(DevStats)) == hipSuccess &&
              // every bucket region empty: a count before the first layout goes to the overflow list
              hipMemset(S.b.cells[0], 0, sizeof(uint4) * (4 * (size_t)c->ntiles + 1)) == hipSuccess &&
              hipMemset(S.b.cells[1], 0, sizeof(uint4) * (4 * (size_t)c->ntiles + 1)) == hipSuccess &&
              hipMemset(S.b.tsum[0], 0, sizeof(uint32_t) * c->ntiles) == hipSuccess &&
              hipMemset(S.b.tsum[1], 0, sizeof(uint32_t) * c->ntiles) == hipSuccess &&
              hipMemset(S.b.ovfn, 0, 2 * sizeof(uint32_t)) == hipSuccess &&
              hipMemset(S.b.scnt, 0, 2 * kXcds * sizeof(uint32_t)) == hipSuccess;
    if (!ok) { stream_free(c); return fail(TRACK_E_DEVICE, "upload failed"); }
    S.m.P = c->P; S.m.L = c->L; S.m.V = c->V; S.m.F = c->F; S.blend = c->blend;
    const float fmax = std::max(camera->fx, camera->fy);
    const double ex = std::max((double)camera->cx + 0.5, (double)camera->width - 0.5 - camera->cx) / camera->fx;
    const double ey = std::max((double)camera->cy + 0.5, (double)camera->height - 0.5 - camera->cy) / camera->fy;
    const double rmax = std::sqrt(1.0 + ex * ex + ey * ey);
    S.c = DevCam{c->W, c->H, tx, ty, camera->fx, camera->fy, camera->cx, camera->cy,
                 (float)((1.0 - 1e-4) / (fmax * rmax))};
    {
        const std::vector<int> order = tile_order(tx, ty, camera->cx, camera->cy);
        if ((int)order.size() != S.b.ntorder || !up(S.b.torder, order.data(), sizeof(int) * order.size())) {
            stream_free(c);
            return fail(TRACK_E_DEVICE, "upload failed");
        }
    }
    int rc;
    if ((rc = stream_set_params(c, params))) { stream_free(c); return rc; }
    std::vector<float> z3(3 * V, 0.0f);
    if ((rc = upload_soa(c->V, S.phi[0], phi0 ? phi0 : z3.data()))) { stream_free(c); return rc; }
    c->v_cur = c->phi_cur = c->phi_prev = 0;
    c->surface_valid = false;
    c->refresh_pose = true;
    return TRACK_OK;
}

// ---------------------------------------------------------------------------
// Batch runner: the slot table, its launches, graphs and kernel timers.
// ---------------------------------------------------------------------------
struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;  // pairs
    size_t used = 0;
    int64_t launches = 0;
    double total_ms = 0.0;
};

struct GraphKey {
    int n, off, kind, skin_first;
    int grid[KK_COUNT_];
    int solve_n, solve_elems, solve_words, ne_pp, ne_l;   // the launch sizes the captured kernels were given
    bool operator==(const GraphKey& o) const {
        if (n != o.n || off != o.off || kind != o.kind || skin_first != o.skin_first) return false;
        if (solve_n != o.solve_n || solve_elems != o.solve_elems || solve_words != o.solve_words || ne_pp != o.ne_pp ||
            ne_l != o.ne_l)
            return false;
        for (int k = 0; k < KK_COUNT_; ++k)
            if (grid[k] != o.grid[k]) return false;
        return true;
    }
};

GraphKey key_of(const Launch& L, int n, int off, int kind) {
    GraphKey k{};
    k.n = n; k.off = off; k.kind = kind; k.skin_first = 1;
    for (int q = 0; q < KK_COUNT_; ++q) k.grid[q] = L.grid[q];
    k.solve_n = L.solve_n; k.solve_elems = L.solve_elems; k.solve_words = L.solve_words;
    k.ne_pp = L.ne_pp; k.ne_l = L.ne_l;
    return k;
}

struct CachedGraph {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
    int seen = 0;         // launches of this key without a graph
    uint64_t last_use = 0;
};

constexpr size_t kMaxGraphs = 64;

struct Runner {
    hipStream_t s = nullptr;
    bool own_stream = false;
    int cap = 0;                       // table entries
    track_allocator alloc{};           // provider of dmem (all null: hipMalloc)
    void* dmem = nullptr;              // dslots and dpre
    Slot* dslots = nullptr;
    int* dpre = nullptr;               // prefix rows of each table window
    Slot* hslots = nullptr;            // pinned; written by the host, read by k_stage
    int* hpre = nullptr;               // pinned
    DevSummary* hsum = nullptr;        // pinned; written by the frame-end kernel
    Slot* hslots_dev = nullptr;        // device views of the pinned buffers
    int* hpre_dev = nullptr;
    DevSummary* hsum_dev = nullptr;
    KernelTimer timers[TRACK_K_COUNT_];
    std::vector<CachedGraph> graphs;
    bool use_graphs = true;
    int capture_after = 0;             // plain launches of a key before it is captured
    uint64_t clock = 0;
    hipEvent_t f0 = nullptr, f1 = nullptr;
};

// prefix rows of the table window starting at entry `off`
inline int pre_offset(int off) { return off * (KK_COUNT_ + 1) * 2; }

int runner_init(Runner& R, int cap, void* hip_stream, const track_allocator* alloc = nullptr) {
    static const bool kernels_ready = prepare_pose_solve() && prepare_normal_eq();
    if (!kernels_ready) return fail(TRACK_E_DEVICE, "pose solve: LDS size attribute refused");
    R.cap = cap;
    if (hip_stream) R.s = (hipStream_t)hip_stream;
    else {
        HIP_TRY(hipStreamCreate(&R.s));
        R.own_stream = true;
    }
    const size_t npre = (size_t)pre_offset(cap) + (size_t)KK_COUNT_ * (cap + 1);
    // the device copy of the table and its prefix rows, one block
    R.alloc = alloc ? *alloc : track_allocator{};
    const size_t slot_bytes = (sizeof(Slot) * cap + 255) & ~size_t(255);
    R.dmem = dev_alloc(R.alloc, slot_bytes + sizeof(int) * npre);
    if (!R.dmem) return fail(TRACK_E_NOMEM, "device allocation failed");
    R.dslots = static_cast<Slot*>(R.dmem);
    R.dpre = reinterpret_cast<int*>(static_cast<char*>(R.dmem) + slot_bytes);
    if (hipHostMalloc(&R.hslots, sizeof(Slot) * cap) != hipSuccess ||
        hipHostMalloc(&R.hpre, sizeof(int) * npre) != hipSuccess ||
        hipHostMalloc(&R.hsum, sizeof(DevSummary) * cap) != hipSuccess)
        return fail(TRACK_E_NOMEM, "pinned allocation failed");
    HIP_TRY(hipHostGetDevicePointer((void**)&R.hslots_dev, R.hslots, 0));
    HIP_TRY(hipHostGetDevicePointer((void**)&R.hpre_dev, R.hpre, 0));
    HIP_TRY(hipHostGetDevicePointer((void**)&R.hsum_dev, R.hsum, 0));
    HIP_TRY(hipEventCreate(&R.f0));
    HIP_TRY(hipEventCreate(&R.f1));
    const char* env = std::getenv("TRACK_NO_GRAPH");
    R.use_graphs = !(env && env[0] == '1');
    return TRACK_OK;
}

void drop_graphs(Runner& R) {
    if (R.s) (void)hipStreamSynchronize(R.s);
    for (auto& g : R.graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    R.graphs.clear();
}

void runner_free(Runner& R) {
    drop_graphs(R);
    for (auto& t : R.timers)
        for (auto e : t.ev) (void)hipEventDestroy(e);
    if (R.f0) (void)hipEventDestroy(R.f0);
    if (R.f1) (void)hipEventDestroy(R.f1);
    dev_free(R.alloc, R.dmem);
    if (R.hslots) (void)hipHostFree(R.hslots);
    if (R.hpre) (void)hipHostFree(R.hpre);
    if (R.hsum) (void)hipHostFree(R.hsum);
    if (R.own_stream && R.s) (void)hipStreamDestroy(R.s);
    R = Runner();
}

bool timing_on(const Runner& R) {
    for (const auto& t : R.timers)
        if (t.on) return true;
    return false;
}

// Kernel timing: a timed pass carries a pair of HIP events that its first and
// last kernels stamp from their own dispatch packets (so the pair spans the
// kernels' execution, not the queue's gaps); launches are then issued
// directly (never from a graph) so that every pair is recorded.
Launch timed(Runner& R, int k, const Launch& L) {
    KernelTimer& t = R.timers[k];
    Launch T = L;
    if (!t.on) return T;
    if (t.used + 2 > t.ev.size()) {
        for (int q = 0; q < 64; ++q) {
            hipEvent_t e;
            // no system-scope fence at the stamps: the pair then times the
            // kernels alone, as a profiler's dispatch trace does
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) == hipSuccess) t.ev.push_back(e);
        }
    }
    if (t.used + 2 <= t.ev.size()) {
        T.t_start = t.ev[t.used];
        T.t_stop = t.ev[t.used + 1];
    }
    return T;
}

void timed_done(Runner& R, int k, const Launch& T) {
    if (T.t_start) R.timers[k].used += 2;
}

// after a stream synchronisation: fold the recorded pairs into totals
void timed_collect(Runner& R) {
    for (auto& t : R.timers) {
        for (size_t q = 0; q + 1 < t.used; q += 2) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, t.ev[q], t.ev[q + 1]) == hipSuccess) {
                t.total_ms += ms;
                t.launches += 1;
            }
        }
        t.used = 0;
    }
}

struct TableEntry {
    Stream* s;
    int flags, iter;
    const float* depth;
    const float* xyz;
};

// Write the table window [off, off + n) and its prefix rows into pinned
// memory and describe the launch; issue_stage() (the launch's first kernel)
// copies them to the device.  The caller synchronises before the window is
// written again.
Launch stage_table(Runner& R, int off, const TableEntry* e, int n) {
    Launch L;
    L.s = R.s;
    int* pre = R.hpre + pre_offset(off);
    for (int k = 0; k < KK_COUNT_; ++k) pre[k * (n + 1)] = 0;
    for (int i = 0; i < n; ++i) {
        Slot S = e[i].s->slot;
        S.v_cur = e[i].s->v_cur;
        S.phi_cur = e[i].s->phi_cur;
        S.phi_prev = e[i].s->phi_prev;
        S.bpar = e[i].s->bpar;
        S.flags = e[i].flags;
        S.iter = e[i].iter;
        S.depth = e[i].depth;
        S.xyz = e[i].xyz;
        S.summary = R.hsum_dev + off + i;
        R.hslots[off + i] = S;
        for (int k = 0; k < KK_COUNT_; ++k) pre[k * (n + 1) + i + 1] = pre[k * (n + 1) + i] + slot_blocks(S, k);
    }
    for (int k = 0; k < KK_COUNT_; ++k) L.grid[k] = pre[k * (n + 1) + n];
    L.solve_n = 16;
    L.solve_elems = 0;
    L.ne_pp = 16;
    L.ne_l = 1;
    L.solve_words = 0;
    bool tree = true;
    for (int i = 0; i < n; ++i) {
        tree = tree && e[i].s->hplan.ok;
        L.solve_elems = std::max(L.solve_elems, e[i].s->hplan.elems);
        L.solve_words = std::max(L.solve_words, e[i].s->hplan.nwords);
        L.solve_n = std::max(L.solve_n, (e[i].s->P + 15) / 16 * 16);
        L.ne_pp = std::max(L.ne_pp, e[i].s->PP);
        L.ne_l = std::max(L.ne_l, e[i].s->L);
    }
    if (!tree) L.solve_elems = L.solve_words = 0;
    L.B.slots = R.dslots + off;
    L.B.pre = R.dpre + pre_offset(off);
    L.B.n = n;
    L.stage_src = R.hslots_dev + off;
    L.stage_pre = R.hpre_dev + pre_offset(off);
    return L;
}

void issue_stage(const Launch& L) {
    launch_stage(L.s, L.stage_src, const_cast<Slot*>(L.B.slots), L.B.n, L.stage_pre, const_cast<int*>(L.B.pre),
                 KK_COUNT_ * (L.B.n + 1));
}

// ---------------------------------------------------------------------------
// The schedule (Section 4): associate, then pose and/or offset steps.
// ---------------------------------------------------------------------------
struct SurfaceState {
    int vsel = 0;          // vertex buffer relative to the launch's start
    int bsel = 0;          // bucket counters of the next count, relative to the launch's start
    int pn = 0;            // offset steps taken since the launch's start
    bool counted = false;  // vsel holds the current surface, counted into the buckets
    bool valid = false;    // vsel holds the current surface
};

void enqueue_associate(Runner& R, const Launch& L, int vsel, int bsel) {
    const Launch T = timed(R, TRACK_K_ASSOC, L);
    launch_associate(T, vsel, bsel);
    timed_done(R, TRACK_K_ASSOC, T);
}

void enqueue_normal_eq(Runner& R, const Launch& L, int gram_mode, int vsel, int pn) {
    {
        const Launch T = timed(R, TRACK_K_NORMAL_EQ, L);
        launch_normal_eq(T, gram_mode, vsel, pn);
        timed_done(R, TRACK_K_NORMAL_EQ, T);
    }
    launch_gram_reduce(L);
}

void enqueue_pose_step(Runner& R, const Launch& L, int fp64, int iter) {
    const Launch T = timed(R, TRACK_K_SOLVE, L);
    launch_pose_solve(T, fp64, iter);
    timed_done(R, TRACK_K_SOLVE, T);
}

void enqueue_skin(Runner& R, const Launch& L, int vsel, int pn, int which, int count, int bsel, int clear_acc) {
    const Launch T = timed(R, TRACK_K_SKIN, L);
    launch_skin(T, vsel, pn, which, count, bsel, 0, clear_acc);
    timed_done(R, TRACK_K_SKIN, T);
}

// Lay out the bucket index of the next count from the surface at the current
// state (forward kinematics first if `fk`): the surface counted alone into
// the other parity (cleared before), its counts laid out into bpar.  Any
// layout gives the same association; this one only keeps the overflow list
// short for the first frame.
void prime_buckets(const Launch& L, bool fk) {
    if (fk) launch_fk(L);
    launch_skin(L, 0, 0, SEL_ALL, SEL_ALL, 1, 1, 0);
    launch_layout(L, 1);
}

// One iteration; `iter` is added to each slot's own iteration index.
// `first`: slots that start here skin and count the surface (the others
// were counted by the step before).  `next`: slots that have another
// iteration after this one -- the kernel that produces their next surface
// counts it into the buckets as well.  Every reader of the buckets and the
// accumulators clears them for the next iteration.  With issue == false only
// the buffer bookkeeping runs (the state a captured launch leaves behind;
// `next` must then be SEL_ALL or SEL_NONE).
void iteration(Runner& R, const Launch& L, const Schedule& sc, bool pose, bool shape, int iter, SurfaceState& st,
               int first, int next, bool issue) {
    const bool more = next != SEL_NONE;
    if (!st.counted) {
        if (issue) enqueue_skin(R, L, st.vsel, st.pn, first, first, st.bsel, 0);
        st.counted = st.valid = true;
    }
    // the association lays out the other parity, which the next count fills
    if (issue) enqueue_associate(R, L, st.vsel, st.bsel);
    st.bsel ^= 1;
    if (pose && issue) {
        enqueue_normal_eq(R, L, sc.gram_mode, st.vsel, st.pn);
        enqueue_pose_step(R, L, sc.pose_fp64, iter);
    }
    if (shape) {
        // re-skin at the new pose into the other vertex buffer, then one
        // offset step, which also skins (and counts) the next surface
        int vn = st.vsel;
        if (pose) {
            vn = st.vsel ^ 1;
            if (issue) enqueue_skin(R, L, vn, st.pn, SEL_ALL, SEL_NONE, st.bsel, 0);
        }
        if (issue) {
            const Launch T = timed(R, TRACK_K_SHAPE, L);
            launch_shape(T, sc.shape_fp64, st.vsel, vn, st.pn, next, st.bsel);
            timed_done(R, TRACK_K_SHAPE, T);
        }
        st.pn += 1;
        st.vsel = more ? vn ^ 1 : vn;
        st.counted = st.valid = more;
    } else if (pose) {
        st.vsel ^= 1;
        if (issue) enqueue_skin(R, L, st.vsel, st.pn, SEL_ALL, next, st.bsel, 1);
        st.counted = more;
        st.valid = true;
    } else {
        if (issue) {
            launch_clear_acc(L);
            launch_bucket_count(L, st.vsel, next, st.bsel);
        }
        st.counted = more;
    }
}

// whole frame of a batch whose slots all start a frame
SurfaceState frame(Runner& R, const Launch& L, const Schedule& sc, bool issue) {
    SurfaceState st;
    if (issue) launch_frame_begin(L);
    for (int t = 0; t < sc.n_iters; ++t)
        iteration(R, L, sc, sc.do_pose[t] != 0, sc.do_shape[t] != 0, t, st, SEL_ALL,
                  t + 1 < sc.n_iters ? SEL_ALL : SEL_NONE, issue);
    if (issue) launch_frame_end(L, sc.first_pose, sc.last_pose);
    return st;
}

// Issue `body`: replay the cached graph of this key, or capture one (once
// the key has been launched `capture_after` times without a graph), or launch
// directly (graphs off, or kernel timing on).  `body` must issue the same
// work for equal keys; what it reads from the slot table is uploaded before
// every launch.
template <class Body>
int run_cached(Runner& R, const GraphKey& key, Body body) {
    ++R.clock;
    if (!R.use_graphs || timing_on(R)) {
        body();
        return TRACK_OK;
    }
    CachedGraph* g = nullptr;
    for (auto& q : R.graphs)
        if (q.key == key) { g = &q; break; }
    if (g && g->exec) {
        g->last_use = R.clock;
        HIP_TRY(hipGraphLaunch(g->exec, R.s));
        return TRACK_OK;
    }
    if (!g) {
        if (R.graphs.size() >= kMaxGraphs) {
            // forget the least recently used key (after its launches finished)
            HIP_TRY(hipStreamSynchronize(R.s));
            size_t lru = 0;
            for (size_t q = 1; q < R.graphs.size(); ++q)
                if (R.graphs[q].last_use < R.graphs[lru].last_use) lru = q;
            if (R.graphs[lru].exec) (void)hipGraphExecDestroy(R.graphs[lru].exec);
            R.graphs.erase(R.graphs.begin() + lru);
        }
        CachedGraph ng;
        ng.key = key;
        R.graphs.push_back(ng);
        g = &R.graphs.back();
    }
    g->last_use = R.clock;
    if (g->seen < R.capture_after) {
        g->seen += 1;
        body();
        return TRACK_OK;
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(R.s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        body();
        e = hipStreamEndCapture(R.s, &graph);
    }
    if (e == hipSuccess) {
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
    }
    if (e != hipSuccess) {
        // no graphs on this stream: launch directly from now on
        (void)hipGetLastError();
        g->exec = nullptr;
        R.use_graphs = false;
        body();
        return TRACK_OK;
    }
    HIP_TRY(hipGraphLaunch(g->exec, R.s));
    return TRACK_OK;
}

const char* lost_reason(int why) {
    switch (why) {
        case 1: return "pose system not positive definite";
        case 2: return "frame has no valid pixels";
        case 3: return "no pixel matched the surface";
        case 4: return "pose diverged";
        case 5: return "energy diverged";
        case 6: return "bucket index overflow (internal error)";
    }
    return "frame rejected";
}

// host record after a frame of stream s: advance or roll back the buffers
void finish_frame(Stream* s, const SurfaceState& st, int status) {
    s->bpar ^= st.bsel;   // every launch of the frame ran, whatever its status
    s->buckets_ready = true;
    if (status == TRACK_OK) {
        s->v_cur ^= st.vsel;
        int q = s->phi_cur;
        for (int k = 0; k < st.pn; ++k) q = phi_next(q, s->phi_prev);
        s->phi_cur = s->phi_prev = q;
        s->surface_valid = st.valid;
        s->refresh_pose = false;
    } else {
        // the pose was restored on the device; the frame-start offsets are
        // untouched in the previous-frame buffer
        s->phi_cur = s->phi_prev;
        s->surface_valid = false;
        s->refresh_pose = true;
    }
}

track_frame_stats to_stats(const DevSummary& d, float ms) {
    track_frame_stats fs{};
    fs.status = d.status;
    fs.n_valid_px = d.n_valid_px;
    fs.n_assoc_px = d.n_assoc_px;
    fs.n_obs_verts = d.n_obs_verts;
    fs.energy_first = d.energy_first;
    fs.energy_last = d.energy_last;
    fs.step_norm_last = d.step_norm_last;
    fs.ms_total = ms;
    return fs;
}

}  // namespace

// ==========================================================================
// Single-stream context: a batch of one.
// ==========================================================================
struct track_ctx {
    Stream st;
    Runner run;
    Schedule sched;
    int gram_mode = 0;
    track_frame_stats last{};
};

namespace {

// stage the context's table (window 0) and issue its upload now
Launch stage_one(track_ctx* c, int flags, const float* depth, const float* xyz) {
    TableEntry e{&c->st, flags, 0, depth, xyz};
    Launch L = stage_table(c->run, 0, &e, 1);
    issue_stage(L);
    return L;
}

// FK (if needed), skin and normals at the current state
int refresh_surface(track_ctx* c) {
    if (c->st.surface_valid) return TRACK_OK;
    Launch L = stage_one(c, 0, nullptr, nullptr);
    if (c->st.refresh_pose) launch_fk(L);
    enqueue_skin(c->run, L, 0, 0, SEL_ALL, SEL_NONE, 0, 0);
    launch_normals(L, 0);
    c->st.surface_valid = true;
    c->st.refresh_pose = false;
    HIP_TRY(hipStreamSynchronize(c->run.s));
    return TRACK_OK;
}

int run_frame(track_ctx* c, const float* depth, const float* xyz) {
    Runner& R = c->run;
    Stream& s = c->st;
    const int flags = kSlotBeginFrame | kSlotEndFrame | (s.refresh_pose ? kSlotRefreshPose : 0);
    if (s.dirty) {  // buckets and accumulators zero, bucket layout from the current surface
        const Launch Lc = stage_one(c, 0, nullptr, nullptr);
        launch_clear(Lc);
        prime_buckets(Lc, s.refresh_pose);
        HIP_TRY(hipStreamSynchronize(R.s));  // before the table window is rewritten
        s.dirty = false;
    }
    TableEntry e{&s, flags, 0, depth, xyz};
    Launch L = stage_table(R, 0, &e, 1);
    const GraphKey key = key_of(L, 1, 0, 0);
    const SurfaceState st = frame(R, L, c->sched, false);
    HIP_TRY(hipEventRecord(R.f0, R.s));
    int rc = run_cached(R, key, [&]() {
        issue_stage(L);
        frame(R, L, c->sched, true);
    });
    if (rc) return rc;
    HIP_TRY(hipEventRecord(R.f1, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    timed_collect(R);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, R.f0, R.f1);
    const DevSummary d = R.hsum[0];
    c->last = to_stats(d, ms);
    finish_frame(&s, st, d.status);
    if (d.status != TRACK_OK) return fail(d.status, lost_reason(d.reason));
    return TRACK_OK;
}

// A frame whose working buffers (frame_scratch_layout) are carved from the
// scratch block at `base` instead of the context's own memory.  Its kernels
// are launched directly, so no graph is instantiated, and nothing is
// allocated.  The block holds whatever the last call on this GPU left, so
// the frame starts by clearing what must start at zero.
int run_frame_noalloc(track_ctx* c, char* base, const float* depth, int32_t on_device) {
    Runner& R = c->run;
    Stream& s = c->st;
    if (timing_on(R)) return fail(TRACK_E_INVALID, "kernel timing is on (its events are created on demand)");
    Slot probe = s.slot;
    const size_t need = frame_scratch_layout(&s, nullptr, probe, nullptr);
    if (need > kScratchBytes)
        return fail(TRACK_E_INVALID, "frame needs " + std::to_string(need) + " bytes of working memory; the "
                    "allocation-free frame has " + std::to_string(kScratchBytes));
    struct Restore {
        Slot& slot;
        const Slot own;
        ~Restore() { slot = own; }
    } restore{s.slot, s.slot};
    float* stage = nullptr;
    frame_scratch_layout(&s, base, s.slot, &stage);
    const float* d = depth;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(stage, depth, sizeof(float) * s.W * s.H, hipMemcpyHostToDevice, R.s));
        d = stage;
    }
    {
        const Launch Lc = stage_one(c, 0, nullptr, nullptr);
        launch_clear(Lc);
        prime_buckets(Lc, s.refresh_pose);
    }
    HIP_TRY(hipStreamSynchronize(R.s));  // before the table window is rewritten
    const int flags = kSlotBeginFrame | kSlotEndFrame | (s.refresh_pose ? kSlotRefreshPose : 0);
    TableEntry e{&s, flags, 0, d, nullptr};
    Launch L = stage_table(R, 0, &e, 1);
    HIP_TRY(hipEventRecord(R.f0, R.s));
    issue_stage(L);
    const SurfaceState st = frame(R, L, c->sched, true);
    HIP_TRY(hipEventRecord(R.f1, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, R.f0, R.f1);
    const DevSummary sum = R.hsum[0];
    c->last = to_stats(sum, ms);
    // the context's own bucket records were not used: keep their parity
    const int bpar = s.bpar;
    const bool ready = s.buckets_ready;
    finish_frame(&s, st, sum.status);
    s.bpar = bpar;
    s.buckets_ready = ready;
    if (sum.status != TRACK_OK) return fail(sum.status, lost_reason(sum.reason));
    return TRACK_OK;
}

void free_ctx(track_ctx* c) {
    if (!c) return;
    runner_free(c->run);
    stream_free(&c->st);
    delete c;
}

}  // namespace

// ==========================================================================
// Serving: many streams, one launch sequence per Gauss-Newton iteration.
// ==========================================================================
namespace {

// deep copy of a model, kept while a stream waits for admission
struct HostModel {
    track_model m{};
    std::vector<int32_t> parent, type, link_joint, faces, skin_link, nbr;
    std::vector<float> axis, offset, rest, skin_w;
    void take(const track_model* s) {
        m = *s;
        parent.assign(s->joint_parent, s->joint_parent + s->n_joints);
        type.assign(s->joint_type, s->joint_type + s->n_joints);
        axis.assign(s->joint_axis, s->joint_axis + 3 * s->n_joints);
        offset.assign(s->joint_offset, s->joint_offset + 7 * s->n_joints);
        link_joint.assign(s->link_joint, s->link_joint + s->n_links);
        rest.assign(s->rest_xyz, s->rest_xyz + 3 * (size_t)s->n_verts);
        faces.assign(s->faces, s->faces + 3 * (size_t)s->n_faces);
        skin_link.assign(s->skin_link, s->skin_link + (size_t)s->n_verts * s->max_infl);
        skin_w.assign(s->skin_w, s->skin_w + (size_t)s->n_verts * s->max_infl);
        if (s->neighbors) nbr.assign(s->neighbors, s->neighbors + 4 * (size_t)s->n_verts);
        m.joint_parent = parent.data(); m.joint_type = type.data(); m.joint_axis = axis.data();
        m.joint_offset = offset.data(); m.link_joint = link_joint.data(); m.rest_xyz = rest.data();
        m.faces = faces.data(); m.skin_link = skin_link.data(); m.skin_w = skin_w.data();
        m.neighbors = s->neighbors ? nbr.data() : nullptr;
    }
    void release() {
        std::vector<int32_t>().swap(faces);
        std::vector<int32_t>().swap(skin_link);
        std::vector<int32_t>().swap(nbr);
        std::vector<float>().swap(rest);
        std::vector<float>().swap(skin_w);
    }
};

struct PendingFrame {
    const float* dev = nullptr;   // caller's device frame, or
    std::vector<float> host;      // a copy of the caller's host frame
    int64_t tag = 0;
};

struct ServerStream {
    int id = -1;
    bool open = false;
    HostModel model;
    track_camera cam{};
    std::vector<double> theta0;
    std::vector<float> phi0;
    size_t bytes = 0;
    Stream* dev = nullptr;        // resident when set
    std::deque<PendingFrame> frames;
    int iter = -1;                // iteration of the frame in progress, -1 = none
};

}  // namespace

struct track_server {
    Runner run;
    Schedule sched;
    track_params params{};
    std::vector<uint8_t> do_pose, do_shape, active;
    int64_t budget = 0, used = 0;
    int max_streams = 0;
    std::vector<ServerStream*> streams;
    std::deque<int> waiting;        // admission queue (stream ids, FIFO)
    std::vector<track_completion> done;
};

namespace {

void server_release(track_server* sv, ServerStream* ss) {
    if (ss->dev) {
        stream_free(ss->dev);
        delete ss->dev;
        ss->dev = nullptr;
        sv->used -= (int64_t)ss->bytes;
    }
}

int server_resident(const track_server* sv) {
    int n = 0;
    for (auto* ss : sv->streams)
        if (ss && ss->dev) ++n;
    return n;
}

// admit waiting streams in arrival order while the budget allows
int server_admit(track_server* sv) {
    while (!sv->waiting.empty()) {
        ServerStream* ss = sv->streams[sv->waiting.front()];
        if (!ss || !ss->open) { sv->waiting.pop_front(); continue; }
        if (sv->used + (int64_t)ss->bytes > sv->budget || server_resident(sv) >= sv->max_streams) break;
        Stream* d = new Stream();
        int rc = stream_create(d, &ss->model.m, &ss->cam, &sv->params, ss->theta0.data(),
                               ss->phi0.empty() ? nullptr : ss->phi0.data(), nullptr);
        if (rc == TRACK_E_NOMEM) { delete d; break; }  // the device is fuller than the budget says
        if (rc) { delete d; return rc; }
        ss->dev = d;
        sv->used += (int64_t)ss->bytes;
        ss->model.release();
        sv->waiting.pop_front();
        // buckets and accumulators start clear, the bucket layout from the
        // stream's first surface
        TableEntry e{d, 0, 0, nullptr, nullptr};
        const Launch Lc = stage_table(sv->run, sv->run.cap - 1, &e, 1);
        issue_stage(Lc);
        launch_clear(Lc);
        prime_buckets(Lc, true);
        HIP_TRY(hipStreamSynchronize(sv->run.s));
        d->dirty = false;
    }
    return TRACK_OK;
}

}  // namespace

// the error record of the calling thread, for the library's other sources
int track_fail_message(int code, const char* msg) { return fail(code, msg); }

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* track_last_error(void) { return g_err.c_str(); }

int track_init(const track_model* model, const track_camera* camera, const track_params* params,
               const double* theta0, const float* phi0, void* hip_stream, const track_allocator* allocator,
               track_ctx** out) {
    g_err.clear();
    if (!out) return fail(TRACK_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = validate_model(model, camera);
    if (rc) return rc;
    if ((rc = validate_params(params, model->n_joints))) return rc;
    if (!theta0) return fail(TRACK_E_INVALID, "theta0 is NULL");
    for (int k = 0; k < model->n_joints; ++k)
        if (!std::isfinite(theta0[k])) return fail(TRACK_E_INVALID, "theta0 not finite");
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(TRACK_E_INVALID, "allocator needs both alloc and free");
    ScaledModel scaled;
    const track_model* mm = scaled.apply(model);
    void* sbase = nullptr;   // the scratch block's address on this device, kept for track_frame_noalloc
    if ((rc = scratch_base(&sbase))) return rc;
    track_ctx* c = new track_ctx();
    if ((rc = runner_init(c->run, 1, hip_stream, allocator))) { free_ctx(c); return rc; }
    if ((rc = stream_create(&c->st, mm, camera, params, theta0, phi0, allocator))) { free_ctx(c); return rc; }
    c->sched.set(params);
    if ((rc = refresh_surface(c))) { free_ctx(c); return rc; }
    *out = c;
    return TRACK_OK;
}

int track_set_params(track_ctx* c, const track_params* p) {
    if (!c) return fail(TRACK_E_INVALID, "ctx is NULL");
    int rc = validate_params(p, c->st.P);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->run.s));
    if ((rc = stream_set_params(&c->st, p))) return rc;
    c->sched.set(p);
    drop_graphs(c->run);
    return TRACK_OK;
}

int track_frame(track_ctx* c, const float* depth, int32_t on_device) {
    if (!c || !depth) return fail(TRACK_E_INVALID, "ctx/depth is NULL");
    const float* d = depth;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(c->st.depth_buf, depth, sizeof(float) * c->st.W * c->st.H, hipMemcpyHostToDevice,
                               c->run.s));
        d = c->st.depth_buf;
    }
    return run_frame(c, d, nullptr);
}

int track_frame_xyz(track_ctx* c, const float* xyz, int32_t on_device) {
    if (!c || !xyz) return fail(TRACK_E_INVALID, "ctx/xyz is NULL");
    const float* d = xyz;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(c->st.xyz_buf, xyz, sizeof(float) * 3 * c->st.W * c->st.H, hipMemcpyHostToDevice,
                               c->run.s));
        d = c->st.xyz_buf;
    }
    return run_frame(c, nullptr, d);
}

int track_frame_noalloc(track_ctx* c, const float* depth, int32_t on_device) {
    if (!c || !depth) return fail(TRACK_E_INVALID, "ctx/depth is NULL");
    void* base = nullptr;
    int rc = scratch_base(&base);
    if (rc) return rc;
    return run_frame_noalloc(c, static_cast<char*>(base), depth, on_device);
}

int track_state(const track_ctx* cc, double* theta, float* phi, float* verts, track_frame_stats* stats) {
    track_ctx* c = const_cast<track_ctx*>(cc);
    if (!c) return fail(TRACK_E_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->run.s));
    const Slot& S = c->st.slot;
    if (theta) HIP_TRY(hipMemcpy(theta, S.theta, sizeof(double) * c->st.P, hipMemcpyDeviceToHost));
    int rc;
    if (phi && (rc = download_soa(c->st.V, S.phi[c->st.phi_cur], phi))) return rc;
    if (verts) {
        if ((rc = refresh_surface(c))) return rc;
        if ((rc = download_v4(c->st.V, S.verts[c->st.v_cur], verts))) return rc;
    }
    if (stats) *stats = c->last;
    return TRACK_OK;
}

int track_reset(track_ctx* c, const double* theta, const float* phi) {
    if (!c || !theta) return fail(TRACK_E_INVALID, "ctx/theta is NULL");
    for (int k = 0; k < c->st.P; ++k)
        if (!std::isfinite(theta[k])) return fail(TRACK_E_INVALID, "theta not finite");
    HIP_TRY(hipStreamSynchronize(c->run.s));
    HIP_TRY(hipMemcpy(c->st.slot.theta, theta, sizeof(double) * c->st.P, hipMemcpyHostToDevice));
    std::vector<float> z3(3 * (size_t)c->st.V, 0.0f);
    int rc;
    if ((rc = upload_soa(c->st.V, c->st.slot.phi[0], phi ? phi : z3.data()))) return rc;
    c->st.phi_cur = c->st.phi_prev = 0;
    c->st.surface_valid = false;
    c->st.refresh_pose = true;
    // the bucket layout follows the surface it was counted from: lay it out
    // again from the new one before the next frame (a far jump would send
    // most vertices to the overflow list)
    c->st.dirty = true;
    return refresh_surface(c);
}

int track_joint_positions(const track_ctx* cc, double* xyz) {
    track_ctx* c = const_cast<track_ctx*>(cc);
    if (!c || !xyz) return fail(TRACK_E_INVALID, "ctx/xyz is NULL");
    const JointTable& t = c->st.hjt;
    std::vector<double> th(t.P);
    HIP_TRY(hipStreamSynchronize(c->run.s));
    HIP_TRY(hipMemcpy(th.data(), c->st.slot.theta, sizeof(double) * t.P, hipMemcpyDeviceToHost));
    // H_{0,j} = H_{0,P(j)} O_j H_j(theta_j), Eq. (1) / (2), then the
    // translation 2 d r* of the dual quaternion r + eps d
    std::vector<double> H(8 * (size_t)t.P);
    for (int j = 0; j < t.P; ++j) {
        double hj[8] = {1, 0, 0, 0, 0, 0, 0, 0};
        const double h = 0.5 * th[j];
        if (t.type[j] == TRACK_HINGE) {
            const double sn = std::sin(h);
            hj[0] = std::cos(h);
            for (int d = 0; d < 3; ++d) hj[1 + d] = sn * t.axis[j][d];
        } else {
            for (int d = 0; d < 3; ++d) hj[5 + d] = h * t.axis[j][d];
        }
        double base[8];
        if (t.parent[j] < 0) std::memcpy(base, t.off[j], sizeof(base));
        else hdq_mul(&H[8 * (size_t)t.parent[j]], t.off[j], base);
        hdq_mul(base, hj, &H[8 * (size_t)j]);
        const double* q = &H[8 * (size_t)j];
        const double rc[4] = {q[0], -q[1], -q[2], -q[3]};
        double tr[4];
        hq_mul(q + 4, rc, tr);
        const double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        for (int d = 0; d < 3; ++d) xyz[3 * j + d] = 2.0 * tr[1 + d] / n2;
    }
    return TRACK_OK;
}

void track_destroy(track_ctx* c) { free_ctx(c); }

int track_kernel_timing(track_ctx* c, int32_t k, int32_t enable) {
    if (!c || k < 0 || k >= TRACK_K_COUNT_) return fail(TRACK_E_INVALID, "bad kernel id");
    HIP_TRY(hipStreamSynchronize(c->run.s));
    timed_collect(c->run);
    c->run.timers[k].on = enable != 0;
    c->run.timers[k].launches = 0;
    c->run.timers[k].total_ms = 0.0;
    return TRACK_OK;
}

int track_kernel_time(track_ctx* c, int32_t k, int64_t* launches, double* total_ms) {
    if (!c || k < 0 || k >= TRACK_K_COUNT_) return fail(TRACK_E_INVALID, "bad kernel id");
    HIP_TRY(hipStreamSynchronize(c->run.s));
    timed_collect(c->run);
    if (launches) *launches = c->run.timers[k].launches;
    if (total_ms) *total_ms = c->run.timers[k].total_ms;
    return TRACK_OK;
}

int track_kernel_bench(track_ctx* c, int32_t k, const float* depth, int32_t reps, double* ms_per_launch) {
    if (!c || !ms_per_launch) return fail(TRACK_E_INVALID, "ctx/ms_per_launch is NULL");
    if (reps < 1 || reps > 100000) return fail(TRACK_E_INVALID, "reps must be in 1..100000");
    if (k != TRACK_K_SKIN && k != TRACK_K_ASSOC && k != TRACK_K_NORMAL_EQ && k != TRACK_K_SOLVE)
        return fail(TRACK_E_INVALID, "kernel cannot be repeated with the same work");
    if (k == TRACK_K_ASSOC || k == TRACK_K_NORMAL_EQ) {
        if (!depth) return fail(TRACK_E_INVALID, "depth is NULL");
        if (!c->st.buckets_ready) return fail(TRACK_E_INVALID, "no tracked frame to repeat");
    }
    Stream& s = c->st;
    Runner& R = c->run;
    HIP_TRY(hipStreamSynchronize(R.s));
    Launch L = stage_one(c, 0, depth, nullptr);
    // the last association read the counters of the other parity, which
    // hold the last count (bpar was laid out by it)
    // (the screen queues of the last association's parity are still full:
    // the repeats start on the other and alternate)
    if (k == TRACK_K_NORMAL_EQ) {  // one association, as inside a frame
        launch_clear_acc(L);
        launch_associate(L, 0, 1, 1);
    }
    HIP_TRY(hipEventRecord(R.f0, R.s));
    for (int r = 0; r < reps; ++r) {
        switch (k) {
            case TRACK_K_SKIN: launch_skin(L, 0, 0, SEL_ALL, SEL_NONE, 0, 0, 0); break;
            case TRACK_K_ASSOC: launch_associate(L, 0, 1, (r & 1) ^ 1); break;
            case TRACK_K_NORMAL_EQ: launch_normal_eq(L, c->sched.gram_mode, 0, 0); break;
            default: launch_pose_solve(L, c->sched.pose_fp64, 0); break;
        }
    }
    HIP_TRY(hipEventRecord(R.f1, R.s));
    HIP_TRY(hipStreamSynchronize(R.s));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, R.f0, R.f1));
    *ms_per_launch = (double)ms / reps;
    // the repeated passes leave partial sums, a moved pose and the like behind
    s.dirty = true;
    s.surface_valid = false;
    s.refresh_pose = true;
    return TRACK_OK;
}

// ---- per-pass access -------------------------------------------------------
int track_dbg_set(track_ctx* c, int32_t buf, const void* host, size_t bytes) {
    if (!c || !host) return fail(TRACK_E_INVALID, "ctx/host is NULL");
    Stream& s = c->st;
    Slot& S = s.slot;
    const size_t V = s.V, N = (size_t)s.W * s.H;
    HIP_TRY(hipStreamSynchronize(c->run.s));
    s.dirty = true;
    switch (buf) {
        case TRACK_BUF_THETA:
            if (bytes != 8 * (size_t)s.P) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(S.theta, host, bytes, hipMemcpyHostToDevice));
            launch_fk(stage_one(c, 0, nullptr, nullptr));
            s.refresh_pose = false;
            break;
        case TRACK_BUF_PHI:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            // keep the previous-frame offsets in their own buffer
            if (s.phi_cur == s.phi_prev) s.phi_cur = phi_next(s.phi_cur, s.phi_prev);
            return upload_soa(s.V, S.phi[s.phi_cur], (const float*)host);
        case TRACK_BUF_PHI_PREV:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            if (s.phi_cur == s.phi_prev) s.phi_prev = phi_next(s.phi_cur, s.phi_prev);
            return upload_soa(s.V, S.phi[s.phi_prev], (const float*)host);
        case TRACK_BUF_VERTS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            s.surface_valid = true;
            return upload_v4(s.V, S.verts[s.v_cur], (const float*)host);
        case TRACK_BUF_NORMALS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return upload_soa(s.V, S.normals, (const float*)host);
        case TRACK_BUF_DEPTH:
            if (bytes != 4 * N) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(s.depth_buf, host, bytes, hipMemcpyHostToDevice));
            s.input_mode = 0;
            break;
        case TRACK_BUF_XYZ:
            if (bytes != 12 * N) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(s.xyz_buf, host, bytes, hipMemcpyHostToDevice));
            s.input_mode = 1;
            break;
        case TRACK_BUF_COUNT:
            if (bytes != 4 * V) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(S.a.cnt, host, bytes, hipMemcpyHostToDevice));
            break;
        case TRACK_BUF_DELTA: {
            // stored as fixed-point sums: count * delta * 2^32 (set COUNT first)
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            std::vector<uint32_t> cnt(V);
            HIP_TRY(hipMemcpy(cnt.data(), S.a.cnt, 4 * V, hipMemcpyDeviceToHost));
            const float* d = (const float*)host;
            std::vector<long long> sm[3];
            for (int q = 0; q < 3; ++q) sm[q].resize(V);
            for (size_t i = 0; i < V; ++i)
                for (int q = 0; q < 3; ++q) sm[q][i] = std::llround((double)d[3 * i + q] * cnt[i] * kFix);
            HIP_TRY(hipMemcpy(S.a.sx, sm[0].data(), 8 * V, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(S.a.sy, sm[1].data(), 8 * V, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(S.a.sz, sm[2].data(), 8 * V, hipMemcpyHostToDevice));
            break;
        }
        default:
            return fail(TRACK_E_INVALID, "buffer cannot be set");
    }
    HIP_TRY(hipStreamSynchronize(c->run.s));
    return TRACK_OK;
}

int track_dbg_get(const track_ctx* cc, int32_t buf, void* host, size_t bytes) {
    track_ctx* c = const_cast<track_ctx*>(cc);
    if (!c || !host) return fail(TRACK_E_INVALID, "ctx/host is NULL");
    Stream& s = c->st;
    const Slot& S = s.slot;
    const size_t V = s.V, N = (size_t)s.W * s.H;
    HIP_TRY(hipStreamSynchronize(c->run.s));
    switch (buf) {
        case TRACK_BUF_THETA:
            if (bytes != 8 * (size_t)s.P) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, S.theta, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_STEP:
            if (bytes != 8 * (size_t)s.P) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, S.step, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_PHI:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_soa(s.V, S.phi[s.phi_cur], (float*)host);
        case TRACK_BUF_PHI_PREV:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_soa(s.V, S.phi[s.phi_prev], (float*)host);
        case TRACK_BUF_VERTS:
        case TRACK_BUF_VERTS_NEW:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_v4(s.V, S.verts[s.v_cur], (float*)host);
        case TRACK_BUF_NORMALS:
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            return download_soa(s.V, S.normals, (float*)host);
        case TRACK_BUF_ASSOC:
            if (bytes != 4 * N) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, S.assoc, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_COUNT:
            if (bytes != 4 * V) return fail(TRACK_E_INVALID, "size");
            HIP_TRY(hipMemcpy(host, S.a.cnt, bytes, hipMemcpyDeviceToHost));
            return TRACK_OK;
        case TRACK_BUF_DELTA: {
            if (bytes != 12 * V) return fail(TRACK_E_INVALID, "size");
            std::vector<uint32_t> cnt(V);
            std::vector<long long> sm[3];
            HIP_TRY(hipMemcpy(cnt.data(), S.a.cnt, 4 * V, hipMemcpyDeviceToHost));
            long long* src[3] = {S.a.sx, S.a.sy, S.a.sz};
            for (int q = 0; q < 3; ++q) {
                sm[q].resize(V);
                HIP_TRY(hipMemcpy(sm[q].data(), src[q], 8 * V, hipMemcpyDeviceToHost));
            }
            float* d = (float*)host;
            for (size_t i = 0; i < V; ++i)
                for (int q = 0; q < 3; ++q)
                    d[3 * i + q] = cnt[i] ? (float)((double)sm[q][i] / ((double)cnt[i] * kFix)) : 0.0f;
            return TRACK_OK;
        }
        case TRACK_BUF_GRAM: {
            const size_t n1 = (size_t)s.P + 1;
            if (bytes != 8 * n1 * n1) return fail(TRACK_E_INVALID, "size");
            std::vector<double> g((size_t)s.PP * s.PP);
            HIP_TRY(hipMemcpy(g.data(), S.gram, 8 * g.size(), hipMemcpyDeviceToHost));
            double* d = (double*)host;
            for (size_t i = 0; i < n1; ++i)
                for (size_t j = 0; j < n1; ++j) d[i * n1 + j] = g[i * s.PP + j];
            return TRACK_OK;
        }
        default:
            return fail(TRACK_E_INVALID, "buffer cannot be read");
    }
}

int track_dbg_run(track_ctx* c, int32_t pass) {
    if (!c) return fail(TRACK_E_INVALID, "ctx is NULL");
    Stream& s = c->st;
    Runner& R = c->run;
    const float* depth = s.input_mode == 0 ? s.depth_buf : nullptr;
    const float* xyz = s.input_mode == 1 ? s.xyz_buf : nullptr;
    HIP_TRY(hipStreamSynchronize(R.s));
    s.dirty = true;
    switch (pass) {
        case TRACK_PASS_SKIN: {
            Launch L = stage_one(c, 0, depth, xyz);
            launch_fk(L);
            enqueue_skin(R, L, 0, 0, SEL_ALL, SEL_NONE, 0, 0);
            launch_normals(L, 0);
            s.surface_valid = true;
            s.refresh_pose = false;
            break;
        }
        case TRACK_PASS_NORMALS:
            launch_normals(stage_one(c, 0, depth, xyz), 0);
            break;
        case TRACK_PASS_ASSOCIATE: {
            // count VERTS in the layout the last association (or priming)
            // left -- none after set-up: every vertex then takes the overflow
            // list -- and associate; the result does not depend on the layout
            Launch L = stage_one(c, 0, depth, xyz);
            launch_clear_acc(L);
            launch_clear_counts(L, 0);
            launch_bucket_count(L, 0, SEL_ALL, 0);
            enqueue_associate(R, L, 0, 0);
            s.bpar ^= 1;
            s.buckets_ready = true;
            break;
        }
        case TRACK_PASS_NORMAL_EQ: {
            Launch L = stage_one(c, 0, depth, xyz);
            launch_fk(L);
            enqueue_normal_eq(R, L, c->sched.gram_mode, 0, 0);
            break;
        }
        case TRACK_PASS_POSE_STEP: {
            Launch L = stage_one(c, kSlotBeginFrame, depth, xyz);
            launch_frame_begin(L);  // clears the status flag
            enqueue_pose_step(R, L, c->sched.pose_fp64, 0);
            s.surface_valid = false;
            break;
        }
        case TRACK_PASS_SHAPE: {
            Launch L = stage_one(c, 0, depth, xyz);
            launch_fk(L);
            enqueue_skin(R, L, 1, 0, SEL_ALL, SEL_NONE, 0, 0);
            {
                const Launch T = timed(R, TRACK_K_SHAPE, L);
                launch_shape(T, c->sched.shape_fp64, 0, 1, 0, SEL_NONE, 0);
                timed_done(R, TRACK_K_SHAPE, T);
            }
            s.v_cur ^= 1;
            s.phi_cur = phi_next(s.phi_cur, s.phi_prev);
            s.surface_valid = false;
            s.refresh_pose = false;
            break;
        }
        default:
            return fail(TRACK_E_INVALID, "unknown pass");
    }
    HIP_TRY(hipStreamSynchronize(R.s));
    timed_collect(R);
    if (pass == TRACK_PASS_POSE_STEP) {
        int st = 0;
        HIP_TRY(hipMemcpy(&st, &s.slot.st->status, sizeof(int), hipMemcpyDeviceToHost));
        if (st == TRACK_E_NOT_PD) return fail(TRACK_E_NOT_PD, "pose system not positive definite");
    }
    return TRACK_OK;
}

// ---- serving ---------------------------------------------------------------
int track_server_create(const track_params* params, int64_t hbm_budget_bytes, int32_t max_streams, void* hip_stream,
                        track_server** out) {
    g_err.clear();
    if (!out) return fail(TRACK_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_streams < 1 || max_streams > 4096) return fail(TRACK_E_INVALID, "max_streams must be in 1..4096");
    if (hbm_budget_bytes <= 0) return fail(TRACK_E_INVALID, "budget must be > 0");
    int rc = validate_params(params, 0);
    if (rc) return rc;
    if (params->active) return fail(TRACK_E_INVALID, "a server takes no per-joint active mask");
    track_server* sv = new track_server();
    sv->params = *params;
    sv->do_pose.assign(params->do_pose, params->do_pose + params->n_iters);
    sv->do_shape.assign(params->do_shape, params->do_shape + params->n_iters);
    sv->params.do_pose = sv->do_pose.data();
    sv->params.do_shape = sv->do_shape.data();
    sv->sched.set(params);
    sv->budget = hbm_budget_bytes;
    sv->max_streams = max_streams;
    // four iteration kinds can share a step; one more entry for clearing a
    // newly admitted stream
    if ((rc = runner_init(sv->run, 4 * max_streams + 1, hip_stream))) {
        runner_free(sv->run);
        delete sv;
        return rc;
    }
    sv->run.capture_after = 2;  // capture a batch shape once it repeats
    *out = sv;
    return TRACK_OK;
}

int track_server_open(track_server* sv, const track_model* model, const track_camera* camera, const double* theta0,
                      const float* phi0, int32_t* stream_id) {
    if (!sv || !stream_id) return fail(TRACK_E_INVALID, "server/stream_id is NULL");
    int rc = validate_model(model, camera);
    if (rc) return rc;
    if (!theta0) return fail(TRACK_E_INVALID, "theta0 is NULL");
    for (int k = 0; k < model->n_joints; ++k)
        if (!std::isfinite(theta0[k])) return fail(TRACK_E_INVALID, "theta0 not finite");
    const size_t bytes = stream_bytes(model, camera);
    if ((int64_t)bytes > sv->budget) return fail(TRACK_E_BUDGET, "stream alone exceeds the memory budget");
    ServerStream* ss = new ServerStream();
    ss->id = (int)sv->streams.size();
    ss->open = true;
    ScaledModel scaled;
    ss->model.take(scaled.apply(model));
    ss->cam = *camera;
    ss->theta0.assign(theta0, theta0 + model->n_joints);
    if (phi0) ss->phi0.assign(phi0, phi0 + 3 * (size_t)model->n_verts);
    ss->bytes = bytes;
    sv->streams.push_back(ss);
    sv->waiting.push_back(ss->id);
    *stream_id = ss->id;
    return server_admit(sv);
}

int track_server_submit(track_server* sv, int32_t id, const float* depth, int32_t on_device, int64_t tag) {
    if (!sv || !depth) return fail(TRACK_E_INVALID, "server/depth is NULL");
    if (id < 0 || id >= (int)sv->streams.size() || !sv->streams[id] || !sv->streams[id]->open)
        return fail(TRACK_E_INVALID, "unknown stream");
    ServerStream* ss = sv->streams[id];
    PendingFrame f;
    f.tag = tag;
    if (on_device) f.dev = depth;
    else f.host.assign(depth, depth + (size_t)ss->cam.width * ss->cam.height);
    ss->frames.push_back(std::move(f));
    return TRACK_OK;
}

int track_server_step(track_server* sv, int32_t* n_completed) {
    if (!sv) return fail(TRACK_E_INVALID, "server is NULL");
    if (n_completed) *n_completed = 0;
    int rc = server_admit(sv);
    if (rc) return rc;
    Runner& R = sv->run;
    const Schedule& sc = sv->sched;
    // streams with work, grouped by the kind of their next iteration
    // (bit 0: pose step, bit 1: offset step)
    std::vector<TableEntry> group[4];
    std::vector<ServerStream*> who[4];
    for (ServerStream* ss : sv->streams) {
        if (!ss || !ss->dev) continue;
        if (ss->iter < 0) {
            if (ss->frames.empty()) continue;
            ss->iter = 0;
            PendingFrame& f = ss->frames.front();
            if (f.dev == nullptr)
                HIP_TRY(hipMemcpyAsync(ss->dev->depth_buf, f.host.data(), sizeof(float) * f.host.size(),
                                       hipMemcpyHostToDevice, R.s));
        }
        const PendingFrame& f = ss->frames.front();
        const int t = ss->iter;
        int flags = 0;
        if (t == 0) flags |= kSlotBeginFrame | (ss->dev->refresh_pose ? kSlotRefreshPose : 0);
        if (t == sc.n_iters - 1) flags |= kSlotEndFrame;
        const int g = (sc.do_pose[t] ? 1 : 0) | (sc.do_shape[t] ? 2 : 0);
        group[g].push_back(TableEntry{ss->dev, flags, t, f.dev ? f.dev : ss->dev->depth_buf, nullptr});
        who[g].push_back(ss);
    }
    int off = 0;
    int nentries = 0;
    for (int g = 0; g < 4; ++g) {
        const int n = (int)group[g].size();
        if (n == 0) continue;
        const bool pose = (g & 1) != 0, shape = (g & 2) != 0;
        Launch L = stage_table(R, off, group[g].data(), n);
        const GraphKey key = key_of(L, n, off, 1 + g);
        rc = run_cached(R, key, [&]() {
            SurfaceState st;
            issue_stage(L);
            launch_frame_begin(L);
            iteration(R, L, sc, pose, shape, 0, st, SEL_BEGIN, SEL_NOT_END, true);
            launch_frame_end(L, sc.first_pose, sc.last_pose);
        });
        if (rc) return rc;
        // the iteration's effect on each stream's buffers (a stream's last
        // iteration prepares no next surface)
        SurfaceState more, last;
        iteration(R, L, sc, pose, shape, 0, more, SEL_ALL, SEL_ALL, false);
        iteration(R, L, sc, pose, shape, 0, last, SEL_ALL, SEL_NONE, false);
        for (ServerStream* ss : who[g]) {
            Stream* d = ss->dev;
            const SurfaceState& it = ss->iter == sc.n_iters - 1 ? last : more;
            d->v_cur ^= it.vsel;
            d->bpar ^= it.bsel;
            if (it.pn) d->phi_cur = phi_next(d->phi_cur, d->phi_prev);
        }
        off += n;
        nentries = off;
    }
    if (nentries == 0) return TRACK_OK;
    HIP_TRY(hipStreamSynchronize(R.s));
    timed_collect(R);
    int ndone = 0;
    off = 0;
    for (int g = 0; g < 4; ++g) {
        for (size_t q = 0; q < who[g].size(); ++q) {
            ServerStream* ss = who[g][q];
            const int t = ss->iter;
            if (t == sc.n_iters - 1) {
                const DevSummary& d = R.hsum[off + q];
                Stream* s = ss->dev;
                // the buffers already advanced; on failure return to the
                // frame-start offsets and redo the surface next frame
                if (d.status == TRACK_OK) {
                    s->phi_prev = s->phi_cur;
                    s->refresh_pose = false;
                } else {
                    s->phi_cur = s->phi_prev;
                    s->refresh_pose = true;
                }
                s->surface_valid = false;
                track_completion cpl{};
                cpl.stream = ss->id;
                cpl.status = d.status;
                cpl.tag = ss->frames.front().tag;
                cpl.stats = to_stats(d, 0.0f);
                sv->done.push_back(cpl);
                ss->frames.pop_front();
                ss->iter = -1;
                ++ndone;
            } else {
                ss->iter = t + 1;
            }
        }
        off += (int)who[g].size();
    }
    if (n_completed) *n_completed = ndone;
    return TRACK_OK;
}

int track_server_poll(track_server* sv, track_completion* out, int32_t max_out, int32_t* n_out) {
    if (!sv || !n_out || (max_out > 0 && !out)) return fail(TRACK_E_INVALID, "bad arguments");
    const int n = std::min<int>(max_out, (int)sv->done.size());
    for (int q = 0; q < n; ++q) out[q] = sv->done[q];
    sv->done.erase(sv->done.begin(), sv->done.begin() + n);
    *n_out = n;
    return TRACK_OK;
}

int track_server_state(track_server* sv, int32_t id, double* theta, float* phi) {
    if (!sv) return fail(TRACK_E_INVALID, "server is NULL");
    if (id < 0 || id >= (int)sv->streams.size() || !sv->streams[id] || !sv->streams[id]->open)
        return fail(TRACK_E_INVALID, "unknown stream");
    ServerStream* ss = sv->streams[id];
    if (!ss->dev) {
        if (theta) std::memcpy(theta, ss->theta0.data(), sizeof(double) * ss->theta0.size());
        if (phi) {
            const size_t n = 3 * (size_t)ss->model.m.n_verts;
            if (ss->phi0.empty()) std::fill(phi, phi + n, 0.0f);
            else std::memcpy(phi, ss->phi0.data(), sizeof(float) * n);
        }
        return TRACK_OK;
    }
    if (ss->iter >= 0) return fail(TRACK_E_INVALID, "stream has a frame in progress");
    HIP_TRY(hipStreamSynchronize(sv->run.s));
    Stream* s = ss->dev;
    if (theta) HIP_TRY(hipMemcpy(theta, s->slot.theta, sizeof(double) * s->P, hipMemcpyDeviceToHost));
    if (phi) return download_soa(s->V, s->slot.phi[s->phi_cur], phi);
    return TRACK_OK;
}

int track_server_close(track_server* sv, int32_t id) {
    if (!sv) return fail(TRACK_E_INVALID, "server is NULL");
    if (id < 0 || id >= (int)sv->streams.size() || !sv->streams[id] || !sv->streams[id]->open)
        return fail(TRACK_E_INVALID, "unknown stream");
    HIP_TRY(hipStreamSynchronize(sv->run.s));
    ServerStream* ss = sv->streams[id];
    server_release(sv, ss);
    delete ss;
    sv->streams[id] = nullptr;
    return server_admit(sv);
}

int track_server_info(track_server* sv, track_server_stats* out) {
    if (!sv || !out) return fail(TRACK_E_INVALID, "server/out is NULL");
    track_server_stats s{};
    for (auto* ss : sv->streams) {
        if (!ss) continue;
        if (ss->dev) ++s.resident;
        else ++s.waiting;
        if (ss->iter >= 0) ++s.frames_in_progress;
        s.frames_pending += (int32_t)ss->frames.size();
    }
    s.bytes_used = sv->used;
    s.bytes_budget = sv->budget;
    *out = s;
    return TRACK_OK;
}

void track_server_destroy(track_server* sv) {
    if (!sv) return;
    if (sv->run.s) (void)hipStreamSynchronize(sv->run.s);
    for (auto* ss : sv->streams) {
        if (!ss) continue;
        server_release(sv, ss);
        delete ss;
    }
    runner_free(sv->run);
    delete sv;
}

}  // extern "C"
