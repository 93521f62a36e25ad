// Precision policies for the transcendental steps of one pair evaluation.
//
// ExactMath evaluates every square root, reciprocal, logarithm and arctangent
// in FP64 (square roots from the hardware estimate and Newton steps, within
// an ulp of the correctly rounded ones).
//
// MixedMath runs them on the FP32 hardware units instead:
//   * sqrt, 1/sqrt and 1/x start from the FP32 estimate and take one Newton
//     step in FP64, which leaves a relative error near 2e-14;
//   * for P0 and P1 fields the arctangent of the sector parts stays in FP32
//     (absolute errors near 1e-7).  A sector part is
//     the whole radial kernel integral times an angular factor, so its
//     sensitivity to the angle is of the size of the integrand and the FP32
//     rounding is not amplified.  For P3 fields the angular factor is
//     multiplied by the field's harmonics about the particle, which carry the
//     extrapolation factor (d_max/width)^3 of the particle-anchored pieces
//     (measured: 3e-6 to 8e-6 on the aspect-ratio-20 covering meshes with
//     FP32 angles), so there the sector angles are evaluated in FP64.
// The logarithm giving H_0 stays in FP64: H_0 enters only the even radial
// terms H_2, H_4, ... (through the p^2 term of the recurrence), so an error in
// it is multiplied by the odd part of the kernel's monomial sum, which does
// not cancel (measured: an FP32 logarithm costs 4e-7 for Wendland C2 and
// 1.5e-5 for C6, the ratio of sum|b_k|/|sum b_k| = 141 and 8.7e3).  The
// recurrences H_c and P_e, the contraction with the kernel coefficients and
// the accumulation stay in FP64.  An edge whose line passes within tau*h of
// the particle (which includes the two edges of a vertex within tau*h) is
// evaluated exactly.
#pragma once

#include <float.h>
#include <math.h>

#include "fastmath.h"

namespace sphbi {

// FP64 1/sqrt(x) and sqrt(x) for finite x > 0 from the hardware estimate and
// two Newton steps (about 10 instructions instead of the 33 of the library's
// correctly rounded 1.0 / sqrt(x); measured within 1 ulp of it).  Arguments
// below 2^-960 are scaled by 2^512 first so that the estimate stays normal.
__device__ inline double rsqrt_nr(double x) {
    const bool tiny = x < 0x1p-960;
    const double xs = tiny ? x * 0x1p512 : x;
    double r = __builtin_amdgcn_rsq(xs);
    double e = fma(-xs * r, r, 1.0);
    r = fma(0.5 * r, e, r);
    e = fma(-xs * r, r, 1.0);
    r = fma(0.5 * r, e, r);
    return tiny ? r * 0x1p256 : r;
}
// The same for arguments that are lengths: x is raised to the smallest
// normal number first (one instruction in place of the scaling), which
// changes nothing for normal x; a subnormal squared length, below 2^-511 h
// as a length, is taken as 2^-511 h.
__device__ inline double rsqrt_len(double x) {
    const double xs = fmax(x, 0x1p-1022);
    double r = __builtin_amdgcn_rsq(xs);
    double e = fma(-xs * r, r, 1.0);
    r = fma(0.5 * r, e, r);
    e = fma(-xs * r, r, 1.0);
    return fma(0.5 * r, e, r);
}
__device__ inline double sqrt_nr(double x) {
    const double r = rsqrt_len(x);
    const double s = x * r;
    return fma(0.5 * r, fma(-s, s, x), s);
}

struct ExactMath {
    // x >= 0 (sqrt_nr(0) = 0: the estimate is taken at the smallest normal)
    __device__ double sqrt_(double x) const { return sqrt_nr(x); }
    __device__ double rsqrt_(double x) const { return rsqrt_nr(x); }
    __device__ double rcp_(double x) const { return 1.0 / x; }
    // angle between the ray to a clipped end at |y| = ay and the circle
    // crossing psi_c (ay >= yc up to rounding, so both arguments are >= 0 up
    // to rounding and the second is > 0)
    __device__ double sector_angle(double p, double ay, double yc) const {
        return atan2_q1(p * (ay - yc), p * p + ay * yc);
    }
    // H_0 = asinh(yB/p) - asinh(yA/p), with asinh(|y|/p) = log((|y| + rho)/p):
    // one quotient and one logarithm whichever signs the ends have
    __device__ double h0(double p, double yA, double yB, double rA, double rB) const {
        const double gA = fabs(yA) + rA, gB = fabs(yB) + rB;
        double num, den, sg;
        if ((yA < 0.0 && yB > 0.0) || (yA > 0.0 && yB < 0.0)) {
            num = gA * gB;
            den = p * p;
            sg = yB > 0.0 ? 1.0 : -1.0;
        } else if (yB != 0.0) {
            num = gB;
            den = gA;
            sg = yB > 0.0 ? 1.0 : -1.0;
        } else {
            num = gA;
            den = p;
            sg = yA > 0.0 ? -1.0 : 1.0;
        }
        return sg * log_pos(div_nr(num, den));
    }
    // length and inverse length of an edge vector
    __device__ void edge_norm(double len2, double &len, double &il) const {
        il = rsqrt_len(len2);
        len = len2 * il;
    }
    // policy for one edge at distance p (in units of h) from the particle
    __device__ ExactMath for_edge(double, double) const { return *this; }
};

// FP32 hardware estimates (one instruction each on gfx950).  Arguments are
// clamped to the smallest normal float: the quantities they serve are lengths
// in units of h, and below 1e-19 h their contribution vanishes anyway.
__device__ inline float rsq_f32(float x) { return __builtin_amdgcn_rsqf(fmaxf(x, FLT_MIN)); }
__device__ inline float rcp_f32(float x) { return __builtin_amdgcn_rcpf(x); }

struct MixedMath {
    bool exact;         // this edge is within tau*h of the particle: evaluate in FP64
    bool fp64_angles;   // sector angles in FP64 (P3 fields)

    __device__ double sqrt_(double x) const {
        if (exact) return sqrt(x);
        const double r = rsq_f32((float)x);
        const double y = x * r;
        return fma(0.5 * r, fma(-y, y, x), y);
    }
    __device__ double rsqrt_(double x) const {
        if (exact) return 1.0 / sqrt(x);
        const double r = rsq_f32((float)x);
        return fma(0.5 * r, fma(-x * r, r, 1.0), r);
    }
    __device__ double rcp_(double x) const {
        if (exact) return 1.0 / x;
        const double r = rcp_f32((float)x);
        return fma(r, fma(-x, r, 1.0), r);
    }
    __device__ double sector_angle(double p, double ay, double yc) const {
        if (exact || fp64_angles) return ExactMath().sector_angle(p, ay, yc);
        return atan2f((float)(p * (ay - yc)), (float)(p * p + ay * yc));
    }
    __device__ double h0(double p, double yA, double yB, double rA, double rB) const {
        if (exact) return ExactMath().h0(p, yA, yB, rA, rB);
        const double gA = fabs(yA) + rA, gB = fabs(yB) + rB;
        double num, den, sg;
        if ((yA < 0.0 && yB > 0.0) || (yA > 0.0 && yB < 0.0)) {
            num = gA * gB;
            den = p * p;
            sg = yB > 0.0 ? 1.0 : -1.0;
        } else if (yB != 0.0) {
            num = gB;
            den = gA;
            sg = yB > 0.0 ? 1.0 : -1.0;
        } else {
            num = gA;
            den = p;
            sg = yA > 0.0 ? -1.0 : 1.0;
        }
        return sg * log_pos(num * rcp_(den));
    }
    __device__ void edge_norm(double len2, double &len, double &il) const {
        il = rsqrt_(len2);
        len = len2 * il;
    }
    // below 1e-15 h the FP32 estimates of 1/p^2 would leave the normal range
    __device__ MixedMath for_edge(double p, double tau) const {
        return MixedMath{p < tau || p < 1e-15, fp64_angles};
    }
};

}  // namespace sphbi
