// C entry points of the CPU oracle (test infrastructure; see oracle.hpp).
// Plain flat arrays in, plain flat arrays out, for ctypes.
#include <cstdint>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.hpp"

#include "capi.h"

static orc::Model to_model(const orc_model_in* in) {
    orc::Model m;
    m.P = in->n_joints; m.L = in->n_links; m.V = in->n_verts; m.F = in->n_faces; m.K = in->max_infl;
    m.parent.assign(in->joint_parent, in->joint_parent + m.P);
    m.type.assign(in->joint_type, in->joint_type + m.P);
    m.link_joint.assign(in->link_joint, in->link_joint + m.L);
    m.faces.assign(in->faces, in->faces + 3 * m.F);
    m.skin_link.assign(in->skin_link, in->skin_link + (size_t)m.V * m.K);
    if (in->neighbors) m.nbr.assign(in->neighbors, in->neighbors + 4 * (size_t)m.V);
    else m.nbr.assign(4 * (size_t)m.V, -1);
    m.axis.assign(in->joint_axis, in->joint_axis + 3 * m.P);
    m.offq.resize(4 * m.P);
    m.offt.resize(3 * m.P);
    for (int j = 0; j < m.P; ++j) {
        for (int c = 0; c < 4; ++c) m.offq[4 * j + c] = in->joint_offset[7 * j + c];
        for (int c = 0; c < 3; ++c) m.offt[3 * j + c] = in->joint_offset[7 * j + 4 + c];
    }
    m.rest.assign(in->rest_xyz, in->rest_xyz + 3 * (size_t)m.V);
    m.skin_w.assign(in->skin_w, in->skin_w + (size_t)m.V * m.K);
    m.blend = in->blend;
    orc::model_derive(m);
    return m;
}

static orc::Camera to_cam(const orc_camera_in* c) { return {c->width, c->height, c->fx, c->fy, c->cx, c->cy}; }

static void put_dq(const orc::DQ<double>& h, double* o) {
    o[0] = h.r.w; o[1] = h.r.x; o[2] = h.r.y; o[3] = h.r.z;
    o[4] = h.d.w; o[5] = h.d.x; o[6] = h.d.y; o[7] = h.d.z;
}

extern "C" {

int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

// World transform of every joint frame (Section 3.1) and every link offset
// H_{l,Delta} (Section 4.2), as 8 doubles (r.w r.x r.y r.z d.w d.x d.y d.z).
int orc_fk(const orc_model_in* in, const double* theta, double* Hj, double* dH) {
    orc::Model m = to_model(in);
    auto H = orc::forward_kinematics<double>(m, theta);
    auto H0 = orc::bind_pose<double>(m);
    auto D = orc::link_deltas(m, H, H0);
    if (Hj) for (int j = 0; j < m.P; ++j) put_dq(H[j], Hj + 8 * j);
    if (dH) for (int l = 0; l < m.L; ++l) put_dq(D[l], dH + 8 * l);
    return 0;
}

// Skinned vertices (Eq. 3, 5) and vertex normals.
int orc_skin(const orc_model_in* in, const double* theta, const double* phi, double* v, double* n) {
    orc::Model m = to_model(in);
    orc::SkinState s = orc::skin_state(m, theta, phi);
    std::copy(s.v.begin(), s.v.end(), v);
    if (n) std::copy(s.n.begin(), s.n.end(), n);
    return 0;
}

// Vertex normals of a given vertex array (float64 [V*3]).
int orc_normals(const orc_model_in* in, const double* v, double* n) {
    orc::Model m = to_model(in);
    orc::vertex_normals(m, v, n);
    return 0;
}

// Forward-mode derivative of the skinned vertices along (dtheta, dphi).
int orc_skin_dual(const orc_model_in* in, const double* theta, const double* dtheta, const double* phi,
                  const double* dphi, double* v, double* dv) {
    orc::Model m = to_model(in);
    std::vector<orc::Dual> th(m.P), ph(3 * (size_t)m.V), out(3 * (size_t)m.V);
    for (int k = 0; k < m.P; ++k) th[k] = orc::Dual(theta[k], dtheta ? dtheta[k] : 0.0);
    for (size_t q = 0; q < ph.size(); ++q) ph[q] = orc::Dual(phi[q], dphi ? dphi[q] : 0.0);
    auto H = orc::forward_kinematics<orc::Dual>(m, th.data());
    auto H0 = orc::bind_pose<orc::Dual>(m);
    auto D = orc::link_deltas(m, H, H0);
    orc::skin(m, D, ph.data(), out.data());
    for (size_t q = 0; q < out.size(); ++q) { v[q] = out[q].v; dv[q] = out[q].d; }
    return 0;
}

// T(H, x) and dT/dH (3x8, row-major) for one dual quaternion.
int orc_transform(const double* H8, const double* x, double* T, double* Jt) {
    orc::DQ<double> H{{H8[0], H8[1], H8[2], H8[3]}, {H8[4], H8[5], H8[6], H8[7]}};
    orc::dq_transform(H, x, T);
    if (Jt) {
        double J[3][8];
        orc::dq_transform_jacobian(H, x, J);
        for (int r = 0; r < 3; ++r) for (int c = 0; c < 8; ++c) Jt[8 * r + c] = J[r][c];
    }
    return 0;
}

// Projective association (Section 4.1); brute != 0 selects the exhaustive
// search, otherwise the 3-D grid.  Exactly one of depth / xyz is non-null.
int orc_associate(const orc_camera_in* c, float tau, const float* v, int32_t V, const float* depth,
                  const float* xyz, int32_t brute, int32_t* a) {
    orc::Camera cam = to_cam(c);
    if (brute) orc::associate_brute(cam, tau, v, V, depth, xyz, a);
    else orc::associate_grid(cam, tau, v, V, depth, xyz, a);
    return 0;
}

int orc_average(const orc_camera_in* c, const float* depth, const float* xyz, const int32_t* a,
                const double* v, int32_t V, int32_t* cnt, double* delta) {
    orc::average_offsets(to_cam(c), depth, xyz, a, v, V, cnt, delta);
    return 0;
}

// Residuals, dense Jacobian rows and normal equations (Eq. 6-8 + prior).
int orc_pose_system(const orc_model_in* in, const double* theta, const double* phi, const double* n,
                    const double* delta, const int32_t* cnt, double lambda_s, double* J, double* r,
                    double* A, double* b, double* rr) {
    orc::Model m = to_model(in);
    orc::PoseSystem ps = orc::pose_system(m, theta, phi, n, delta, cnt, lambda_s);
    if (J) std::copy(ps.J.begin(), ps.J.end(), J);
    if (r) std::copy(ps.r.begin(), ps.r.end(), r);
    if (A) std::copy(ps.A.begin(), ps.A.end(), A);
    if (b) std::copy(ps.b.begin(), ps.b.end(), b);
    if (rr) *rr = ps.rr;
    return 0;
}

int orc_prior_weights(const orc_model_in* in, double* out) {
    orc::Model m = to_model(in);
    auto s = orc::prior_weights(m);
    std::copy(s.begin(), s.end(), out);
    return 0;
}

int orc_lm_solve(int32_t P, const double* A, const double* b, double lambda_k, const uint8_t* active,
                 double* x) {
    return orc::lm_solve(P, A, b, lambda_k, active, x);
}

int orc_shape_step(const orc_model_in* in, const double* theta, const double* phi, const double* phi_prev,
                   const double* n, const double* delta, const int32_t* cnt, double lphi, double lnbr,
                   double lt, double lw, double* phi_out) {
    orc::Model m = to_model(in);
    orc::ShapeArgs s{theta, phi, phi_prev, n, delta, cnt, lphi, lnbr, lt, lw};
    orc::shape_step(m, s, phi_out);
    return 0;
}

int orc_shape_step_literal(const orc_model_in* in, const double* theta, const double* phi, const double* phi_prev,
                           const double* n, const double* delta, const int32_t* cnt, double lphi, double lnbr,
                           double lw, double* phi_out) {
    orc::Model m = to_model(in);
    orc::ShapeArgs s{theta, phi, phi_prev, n, delta, cnt, lphi, lnbr, 0.0, lw};
    orc::shape_step_literal(m, s, phi_out);
    return 0;
}

// One frame.  stats_i = {status, n_valid_px, n_assoc_px, n_obs_verts},
// stats_d = {energy_first, energy_last, step_norm_last}.
int orc_track_frame(const orc_model_in* in, const orc_camera_in* c, const orc_params_in* p, double* theta,
                    double* phi, double* phi_prev, const float* depth, const float* xyz, int32_t* stats_i,
                    double* stats_d, double* energies, int32_t* assoc_first, const int32_t* assoc_in) {
    orc::Model m = to_model(in);
    orc::Params prm;
    prm.tau = p->tau;
    prm.n_iters = p->n_iters;
    prm.do_pose.assign(p->do_pose, p->do_pose + p->n_iters);
    prm.do_shape.assign(p->do_shape, p->do_shape + p->n_iters);
    if (p->active) prm.active.assign(p->active, p->active + m.P);
    prm.lambda_k = p->lambda_k; prm.lambda_s = p->lambda_s; prm.lambda_phi = p->lambda_phi;
    prm.lambda_nbr = p->lambda_nbr; prm.lambda_t = p->lambda_t; prm.lambda_w = p->lambda_w;
    orc::FrameStats st{};
    int rc = orc::track_frame(m, to_cam(c), prm, theta, phi, phi_prev, depth, xyz, &st, energies, assoc_first, assoc_in);
    if (stats_i) { stats_i[0] = st.status; stats_i[1] = st.n_valid_px; stats_i[2] = st.n_assoc_px; stats_i[3] = st.n_obs_verts; }
    if (stats_d) { stats_d[0] = st.energy_first; stats_d[1] = st.energy_last; stats_d[2] = st.step_norm_last; }
    return rc;
}

}  // extern "C"
