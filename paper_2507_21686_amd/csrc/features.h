// Canonical features of one (particle, triangle) pair for the learned
// surrogate, in the support-normalised particle frame (Sec. 2, transform C).
//
//   * counter-clockwise vertex order (the integrals do not depend on it);
//   * cyclic shift so the vertex nearest the particle comes first (lowest
//     index on ties);
//   * rotation about the particle putting that vertex on the +x axis
//     (identity when it coincides with the particle);
//   * features 0-5: the rotated vertices; 6: vertices with |nu| <= 1, over 3;
//     7: edges whose segment meets the circle |nu| = 1, over 3.
// Every decision is taken in FP64 without fused multiply-adds, so it is
// reproducible bit for bit by a plain evaluation of the same formulas.
#pragma once

#include <math.h>

namespace sphbi {

__host__ __device__ inline bool segment_meets_circle(double a0, double a1, double b0, double b1) {
#pragma clang fp contract(off)
    const double da = a0 * a0 + a1 * a1;
    const double db = b0 * b0 + b1 * b1;
    if ((da <= 1.0) != (db <= 1.0)) return true;
    if (da <= 1.0) return false;                       // both inside
    const double ex = b0 - a0, ey = b1 - a1;           // both outside: closest point inside?
    const double L2 = ex * ex + ey * ey;
    if (L2 == 0.0) return false;
    const double t = -(a0 * ex + a1 * ey) / L2;
    if (t <= 0.0 || t >= 1.0) return false;
    const double cx = a0 + t * ex, cy = a1 + t * ey;
    return cx * cx + cy * cy < 1.0;
}

// x, y: particle; v: vertex coordinates x0 y0 x1 y1 x2 y2 (world units).
// f[8]: features; (c, s): cosine and sine of the frame rotation.
__host__ __device__ inline void pair_features(double x, double y, const double *v, double invh, float *f,
                                              double &c, double &s) {
#pragma clang fp contract(off)
    double vx[3], vy[3];
    for (int k = 0; k < 3; ++k) {
        vx[k] = (v[2 * k] - x) * invh;
        vy[k] = (v[2 * k + 1] - y) * invh;
    }
    const double area2 = (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]);
    if (area2 < 0.0) {
        double t = vx[1]; vx[1] = vx[2]; vx[2] = t;
        t = vy[1]; vy[1] = vy[2]; vy[2] = t;
    }
    double d2[3];
    for (int k = 0; k < 3; ++k) d2[k] = vx[k] * vx[k] + vy[k] * vy[k];
    int first = 0;
    if (d2[1] < d2[first]) first = 1;
    if (d2[2] < d2[first]) first = 2;
    double ux[3], uy[3], ud[3];
    for (int k = 0; k < 3; ++k) {
        const int j = (first + k) % 3;
        ux[k] = vx[j];
        uy[k] = vy[j];
        ud[k] = d2[j];
    }
    const double r = sqrt(ud[0]);
    c = 1.0;
    s = 0.0;
    if (r > 0.0) {
        c = ux[0] / r;
        s = uy[0] / r;
    }
    int inside = 0, cross = 0;
    for (int k = 0; k < 3; ++k) {
        f[2 * k] = (float)(c * ux[k] + s * uy[k]);
        f[2 * k + 1] = (float)(c * uy[k] - s * ux[k]);
        inside += ud[k] <= 1.0 ? 1 : 0;
        const int j = k == 2 ? 0 : k + 1;
        cross += segment_meets_circle(ux[k], uy[k], ux[j], uy[j]) ? 1 : 0;
    }
    f[6] = (float)(inside / 3.0);
    f[7] = (float)(cross / 3.0);
}

}  // namespace sphbi
