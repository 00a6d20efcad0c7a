// C views of the oracle's inputs, shared by its entry points (test
// infrastructure; see oracle.hpp).
#pragma once
#include <cstdint>

extern "C" {

typedef struct {
    int32_t n_joints;
    const int32_t* joint_parent;
    const int32_t* joint_type;
    const float* joint_axis;    // [P*3]
    const float* joint_offset;  // [P*7] quaternion (w,x,y,z), translation
    int32_t n_links;
    const int32_t* link_joint;
    int32_t n_verts;
    const float* rest_xyz;      // [V*3]
    int32_t n_faces;
    const int32_t* faces;       // [F*3]
    int32_t max_infl;
    const int32_t* skin_link;   // [V*K]
    const float* skin_w;        // [V*K]
    const int32_t* neighbors;   // [V*4]
    int32_t blend;              // 0 dual-quaternion blend, 1 linear blend of the links' transforms
} orc_model_in;

typedef struct { int32_t width, height; float fx, fy, cx, cy; } orc_camera_in;

typedef struct {
    float tau;
    int32_t n_iters;
    const uint8_t* do_pose;
    const uint8_t* do_shape;
    const uint8_t* active;
    double lambda_k, lambda_s, lambda_phi, lambda_nbr, lambda_t, lambda_w;
} orc_params_in;

}  // extern "C"
