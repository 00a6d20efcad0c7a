/*
 * Depth rendering for the synthetic workloads.
 *
 * This file produces observations, not tracker arithmetic: it z-buffers a
 * camera-space triangle mesh into a pinhole depth image (the stand-in for the
 * depth sensor the paper uses, Section 5.1) and splats camera-space points
 * into an organised point cloud (the "every point is a pixel" layout of
 * Section 4.1).  Pixel centres sit at integer (u, v); a camera-space point
 * (x, y, z) maps to u = fx*x/z + cx, v = fy*y/z + cy.
 *
 * Built with gcc as a plain shared object; called through ctypes.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* Depth of the plane through a,b,c along the ray through pixel (u, v); the
 * ray direction is ((u-cx)/fx, (v-cy)/fy, 1), so the returned t is z. */
static double ray_plane_z(const double *a, const double *b, const double *c,
                          double dx, double dy) {
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                   e1[0] * e2[1] - e1[1] * e2[0]};
    double den = n[0] * dx + n[1] * dy + n[2];
    if (fabs(den) < 1e-300) return -1.0;
    return (n[0] * a[0] + n[1] * a[1] + n[2] * a[2]) / den;
}

/* Rasterise triangles into a z-buffer.  depth[h*W+w] holds the nearest z
 * (metres) or +INFINITY where nothing was drawn; it is initialised here.
 * Triangles with any vertex at z <= znear are skipped.  Returns the number of
 * covered pixels. */
int synth_raster_depth(const float *xyz, int32_t n_verts, const int32_t *faces,
                       int32_t n_faces, int32_t W, int32_t H, double fx,
                       double fy, double cx, double cy, double znear,
                       float *depth) {
    for (int64_t i = 0; i < (int64_t)W * H; ++i) depth[i] = INFINITY;
    for (int32_t f = 0; f < n_faces; ++f) {
        double P[3][3], uv[3][2];
        int ok = 1;
        for (int k = 0; k < 3; ++k) {
            int32_t vi = faces[3 * f + k];
            if (vi < 0 || vi >= n_verts) return -1;
            for (int d = 0; d < 3; ++d) P[k][d] = xyz[3 * (int64_t)vi + d];
            if (P[k][2] <= znear) { ok = 0; break; }
            uv[k][0] = fx * P[k][0] / P[k][2] + cx;
            uv[k][1] = fy * P[k][1] / P[k][2] + cy;
        }
        if (!ok) continue;
        double umin = fmin(uv[0][0], fmin(uv[1][0], uv[2][0]));
        double umax = fmax(uv[0][0], fmax(uv[1][0], uv[2][0]));
        double vmin = fmin(uv[0][1], fmin(uv[1][1], uv[2][1]));
        double vmax = fmax(uv[0][1], fmax(uv[1][1], uv[2][1]));
        int u0 = (int)ceil(umin), u1 = (int)floor(umax);
        int v0 = (int)ceil(vmin), v1 = (int)floor(vmax);
        if (u0 < 0) u0 = 0;
        if (v0 < 0) v0 = 0;
        if (u1 > W - 1) u1 = W - 1;
        if (v1 > H - 1) v1 = H - 1;
        if (u0 > u1 || v0 > v1) continue;
        /* signed doubled area in the image plane */
        double area = (uv[1][0] - uv[0][0]) * (uv[2][1] - uv[0][1]) -
                      (uv[2][0] - uv[0][0]) * (uv[1][1] - uv[0][1]);
        if (fabs(area) < 1e-12) continue;
        for (int v = v0; v <= v1; ++v) {
            for (int u = u0; u <= u1; ++u) {
                double w0 = (uv[2][0] - uv[1][0]) * (v - uv[1][1]) -
                            (uv[2][1] - uv[1][1]) * (u - uv[1][0]);
                double w1 = (uv[0][0] - uv[2][0]) * (v - uv[2][1]) -
                            (uv[0][1] - uv[2][1]) * (u - uv[2][0]);
                double w2 = (uv[1][0] - uv[0][0]) * (v - uv[0][1]) -
                            (uv[1][1] - uv[0][1]) * (u - uv[0][0]);
                int inside = (area > 0) ? (w0 >= 0 && w1 >= 0 && w2 >= 0)
                                        : (w0 <= 0 && w1 <= 0 && w2 <= 0);
                if (!inside) continue;
                double z = ray_plane_z(P[0], P[1], P[2], (u - cx) / fx,
                                       (v - cy) / fy);
                if (!(z > znear)) continue;
                float zf = (float)z;
                int64_t idx = (int64_t)v * W + u;
                if (zf < depth[idx]) depth[idx] = zf;
            }
        }
    }
    int covered = 0;
    for (int64_t i = 0; i < (int64_t)W * H; ++i) covered += isfinite(depth[i]) ? 1 : 0;
    return covered;
}

/* Splat points into an organised point cloud.  For each point with
 * keep[i] != 0 and z > znear whose rounded projection floor(u+0.5),
 * floor(v+0.5) lands in the image, the nearest point (smallest z, then the
 * smallest index) wins the pixel.  out_xyz[(h*W+w)*3 + d] receives the point
 * itself; pixels no point reached get (0, 0, 0).  out_id receives the point's
 * index or -1.  Returns the number of filled pixels. */
int synth_splat_points(const float *xyz, const uint8_t *keep, int32_t n,
                       int32_t W, int32_t H, double fx, double fy, double cx,
                       double cy, double znear, float *out_xyz,
                       int32_t *out_id) {
    for (int64_t i = 0; i < (int64_t)W * H; ++i) {
        out_id[i] = -1;
        out_xyz[3 * i + 0] = out_xyz[3 * i + 1] = out_xyz[3 * i + 2] = 0.0f;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (keep && !keep[i]) continue;
        double x = xyz[3 * (int64_t)i], y = xyz[3 * (int64_t)i + 1],
               z = xyz[3 * (int64_t)i + 2];
        if (!(z > znear)) continue;
        int u = (int)floor(fx * x / z + cx + 0.5);
        int v = (int)floor(fy * y / z + cy + 0.5);
        if (u < 0 || v < 0 || u >= W || v >= H) continue;
        int64_t idx = (int64_t)v * W + u;
        int32_t cur = out_id[idx];
        if (cur < 0 || z < xyz[3 * (int64_t)cur + 2]) {
            out_id[idx] = i;
        }
    }
    int filled = 0;
    for (int64_t i = 0; i < (int64_t)W * H; ++i) {
        int32_t id = out_id[i];
        if (id < 0) continue;
        ++filled;
        for (int d = 0; d < 3; ++d) out_xyz[3 * i + d] = xyz[3 * (int64_t)id + d];
    }
    return filled;
}
