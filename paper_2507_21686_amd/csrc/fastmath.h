// FP64 arctangent and logarithm for the argument ranges of the pair
// evaluation, from their series with fitted coefficients (fit_series.py
// generates them).  The general library routines handle every quadrant,
// sign, infinity and subnormal; here the arguments are known to be finite
// with y >= 0, x > 0 (sector angles) and x > 0 normal (the radial term H_0),
// which removes most of their work.  Accuracy: a few units in the last place
// (measured against the C library on 2e7 random arguments: 4 and 3.4 ulp).
#pragma once

#include <math.h>

namespace sphbi {

// An FP64 constant cannot be an instruction literal on this target.  Written
// inline, each coefficient would be materialised once in a vector register
// pair and kept for the whole loop it is hoisted out of; under register
// pressure the compiler then spills it and reloads it from scratch memory
// inside the polynomial.  sconst() hands the constant over through an opaque
// scalar-register operand at the point of use, so it costs two scalar moves
// (issued beside the vector work; the hazard check adds a one-cycle wait after
// the empty asm) and no vector register.  Measured on the cubic-field forward
// kernel: 238 vector registers and no spills, against 256 and 68 bytes of
// scratch spills per lane with plain constants; with the compiler's machine
// loop-invariant code motion off, plain constants spill no more but cost a
// vector move at each use (333 against 141 vector moves in the kernel).
//
// A translation unit that defines SPHBI_PLAIN_CONSTANTS before including this
// header gets plain constants instead.  The adjoint's unit for constant and
// cubic fields does: its kernels run one wave per SIMD, where the operand form
// only adds instructions (0.608 against 0.589 ms on the C4/P3 differentiation
// workload, bit-identical results).  An earlier version of that adjoint gave
// wrong moments in its fully unrolled cubic instantiation with the operand
// form; the current one passes every adjoint parity test with either form,
// and the cause of the earlier failure was not found.  lit() now hands only
// compile-time constants to the operand, so a lane-varying value can never
// be read from a single lane.
#ifdef SPHBI_PLAIN_CONSTANTS
__device__ inline double sconst(double c) { return c; }
#else
__device__ inline double sconst(double c) {
    asm volatile("" : "+s"(c));
    return c;
}
#endif

// a / b from the hardware reciprocal estimate (v_rcp_f64, relative error
// 4.6e-8 over the normal range), two Newton steps on the reciprocal and one
// correction of the quotient: 8 instructions instead of the 10 and a hazard
// wait of the IEEE division sequence, whose scaling steps handle the over-
// and underflowing operands that the callers here exclude (b and a / b
// normal).  Measured on 4M operand pairs with b over every normal exponent:
// equal to the correctly rounded quotient in every case.
__device__ inline double div_nr(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

// atan(y / x) for y >= 0, x > 0.  After swapping so that the ratio is at
// most 1, the identity atan(t) = pi/4 + atan((t - 1)/(t + 1)) brings it to
// |u| <= tan(pi/8) with one division, where atan(u) = u + u^3 P(u^2)
// (P of degree 9, relative error 7e-17).
__device__ inline double atan2_q1(double y, double x) {
    const bool swap = y > x;
    const double num = swap ? x : y, den = swap ? y : x;
    const bool big = num > sconst(0.41421356237309503) * den;
    const double u = div_nr(big ? num - den : num, big ? num + den : den);
    const double s = u * u;
    double p = sconst(0.02114282795405936);
    p = fma(p, s, sconst(-0.043486934438068184));
    p = fma(p, s, sconst(0.05688583712710041));
    p = fma(p, s, sconst(-0.06640281421077107));
    p = fma(p, s, sconst(0.07689959311291694));
    p = fma(p, s, sconst(-0.09090773515721326));
    p = fma(p, s, sconst(0.11111106200822037));
    p = fma(p, s, sconst(-0.1428571418151725));
    p = fma(p, s, sconst(0.1999999999886241));
    p = fma(p, s, sconst(-0.33333333333328474));
    double a = fma(u * s, p, u);
    if (big) a += sconst(0.7853981633974483);
    return swap ? sconst(1.5707963267948966) - a : a;
}

// log(x) for finite normal x > 0: x = m 2^e with m in [1/sqrt 2, sqrt 2),
// log m = 2 atanh(s) = 2 s + s^3 Q(s^2), s = (m - 1)/(m + 1) (Q of degree 7,
// relative error 7e-19), and e ln 2 with ln 2 split so that e ln2_hi is exact.
__device__ inline double log_pos(double x) {
    int e;
    double m = frexp(x, &e);                       // m in [1/2, 1)
    if (m < sconst(0.7071067811865476)) {
        m *= 2.0;
        e -= 1;
    }
    const double s = div_nr(m - 1.0, m + 1.0);
    const double s2 = s * s;
    double q = sconst(0.1326226214625569);
    q = fma(q, s2, sconst(0.13248744435029344));
    q = fma(q, s2, sconst(0.1538716181755671));
    q = fma(q, s2, sconst(0.18181773715830785));
    q = fma(q, s2, sconst(0.22222222677235373));
    q = fma(q, s2, sconst(0.28571428568816837));
    q = fma(q, s2, sconst(0.400000000000075));
    q = fma(q, s2, sconst(0.6666666666666666));
    const double lm = fma(s * s2, q, 2.0 * s);
    const double de = (double)e;
    return fma(de, sconst(0.6931471803691238), fma(de, sconst(1.9082149292705877e-10), lm));
}


}  // namespace sphbi
