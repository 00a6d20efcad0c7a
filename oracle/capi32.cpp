// Float32 instantiation of the oracle's frame (test infrastructure; see
// oracle.hpp): the same source with its scalar set to float, in namespace
// orc32, for the CPU timing baseline at the precision the GPU path computes
// in.  Reference values and pins always come from the float64 instantiation.
#include <cstdint>
#include <vector>
#define ORC_REAL float
#define ORC_NS orc32
#include "oracle.hpp"
#include "capi.h"

static orc32::Model to_model32(const orc_model_in* in) {
    orc32::Model m;
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
    orc32::model_derive(m);
    return m;
}

extern "C" {

// One frame in float32 (the state converted from and back to float64 at the
// boundary).  stats_i = {status, n_valid_px, n_assoc_px, n_obs_verts}.
int orc32_track_frame(const orc_model_in* in, const orc_camera_in* c, const orc_params_in* p, double* theta,
                      double* phi, double* phi_prev, const float* depth, const float* xyz, int32_t* stats_i) {
    orc32::Model m = to_model32(in);
    orc32::Params prm;
    prm.tau = p->tau;
    prm.n_iters = p->n_iters;
    prm.do_pose.assign(p->do_pose, p->do_pose + p->n_iters);
    prm.do_shape.assign(p->do_shape, p->do_shape + p->n_iters);
    if (p->active) prm.active.assign(p->active, p->active + m.P);
    prm.lambda_k = (float)p->lambda_k; prm.lambda_s = (float)p->lambda_s; prm.lambda_phi = (float)p->lambda_phi;
    prm.lambda_nbr = (float)p->lambda_nbr; prm.lambda_t = (float)p->lambda_t; prm.lambda_w = (float)p->lambda_w;
    std::vector<float> th(theta, theta + m.P), ph(phi, phi + 3 * (size_t)m.V), pp(phi_prev, phi_prev + 3 * (size_t)m.V);
    orc32::FrameStats st{};
    const orc32::Camera cam{c->width, c->height, c->fx, c->fy, c->cx, c->cy};
    int rc = orc32::track_frame(m, cam, prm, th.data(), ph.data(), pp.data(), depth, xyz, &st, nullptr, nullptr);
    for (int k = 0; k < m.P; ++k) theta[k] = th[k];
    for (size_t q = 0; q < ph.size(); ++q) { phi[q] = ph[q]; phi_prev[q] = pp[q]; }
    if (stats_i) { stats_i[0] = st.status; stats_i[1] = st.n_valid_px; stats_i[2] = st.n_assoc_px; stats_i[3] = st.n_obs_verts; }
    return rc;
}

}  // extern "C"
