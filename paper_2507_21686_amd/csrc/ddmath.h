// Double-double arithmetic (an unevaluated sum hi + lo of two doubles,
// |lo| <= ulp(hi)/2, about 106 bits) and the precision policy DDMath for the
// ill-conditioned pairs of the forward integrals.
//
// The closed form of a pair sums particle-anchored pieces that cover the
// region between the particle and the triangle, and expands the field in
// harmonics about the particle.  For a thin triangle seen from a particle
// beside it the pieces and the harmonic terms are larger than their sum by
// the extrapolation factor (d_max / width)^order, so FP64 loses that many
// digits.  The same pair evaluated with every step in double-double (the
// frame transform of the exact input doubles, the field preparation, the
// shift to the particle, the radial recurrences, the angles, the logarithm
// and the contraction) keeps about 32 - log10(factor) digits, so its result
// rounded to FP64 is accurate to the last bits for any factor below 1e15.
//
// The error-free transformations are Knuth's TwoSum, Dekker's FastTwoSum and
// the fused-multiply-add form of TwoProduct; the compound operations follow
// the usual double-double algorithms (addition with one TwoSum of the high
// parts, multiplication with the cross terms, division by two correction
// steps, square root by one Newton step).  The addition is the short form:
// its error is a few units of 2^-106 of |a| + |b| rather than of the sum, so a
// single addition that cancels by a factor F keeps about 32 - log10(F)
// digits -- the same budget as the conditioning above, and well inside it
// (the longer form, a second TwoSum of the low parts, cost a sixth more time
// in the refinement pass and changed no result by more than 1e-22).  They rely on every product and sum being
// rounded on its own exactly as written: a product fused into a following
// addition (FP contraction, on by default for device code) breaks the error
// terms -- measured on gfx950: products and quotients then carry 1e-16
// relative errors instead of 1e-32.  Every function body here therefore
// turns contraction off (SPHBI_DD_EXACT); the pragma marks the operations of
// that body, so they stay unfused after inlining into any caller.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#define SPHBI_DD_EXACT _Pragma("clang fp contract(off)")

namespace sphbi {

// The type and its operators live in a namespace of their own, so that the
// overloads of fabs, fma, copysign and ldexp are found for double-double
// arguments (by argument-dependent lookup) without hiding the FP64 library
// functions from code in namespace sphbi.
namespace ddarith {

struct dd {
    double hi, lo;
    __host__ __device__ constexpr dd() : hi(0.0), lo(0.0) {}
    __host__ __device__ constexpr dd(double x) : hi(x), lo(0.0) {}
    __host__ __device__ constexpr dd(double h, double l) : hi(h), lo(l) {}
    __host__ __device__ explicit operator double() const { return hi + lo; }
};

}  // namespace ddarith
using ddarith::dd;

// ---- error-free transformations
__host__ __device__ inline dd two_sum(double a, double b) {
    SPHBI_DD_EXACT
    const double s = a + b;
    const double bb = s - a;
    return dd(s, (a - (s - bb)) + (b - bb));
}
__host__ __device__ constexpr dd fast_two_sum(double a, double b) {   // |a| >= |b| or a == 0
    SPHBI_DD_EXACT
    return dd(a + b, b - ((a + b) - a));
}
__host__ __device__ inline dd two_prod(double a, double b) {
    SPHBI_DD_EXACT
    const double p = a * b;
    return dd(p, fma(a, b, -p));
}

namespace ddarith {

// ---- arithmetic
__host__ __device__ inline dd operator-(const dd &a) {
    SPHBI_DD_EXACT
    return dd(-a.hi, -a.lo);
}
__host__ __device__ inline dd operator+(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    dd s = two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return fast_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd operator+(const dd &a, double b) {
    SPHBI_DD_EXACT
    dd s = two_sum(a.hi, b);
    s.lo += a.lo;
    return fast_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd operator+(double a, const dd &b) {
    SPHBI_DD_EXACT
    return b + a;
}
__host__ __device__ inline dd operator-(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return a + (-b);
}
__host__ __device__ inline dd operator-(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a + (-b);
}
__host__ __device__ inline dd operator-(double a, const dd &b) {
    SPHBI_DD_EXACT
    return (-b) + a;
}
// (the cross terms are folded into the error term with explicit fused
// multiply-adds: one rounding each instead of two)
__host__ __device__ inline dd operator*(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    dd p = two_prod(a.hi, b.hi);
    p.lo = ::fma(a.hi, b.lo, ::fma(a.lo, b.hi, p.lo));
    return fast_two_sum(p.hi, p.lo);
}
__host__ __device__ inline dd operator*(const dd &a, double b) {
    SPHBI_DD_EXACT
    dd p = two_prod(a.hi, b);
    p.lo = ::fma(a.lo, b, p.lo);
    return fast_two_sum(p.hi, p.lo);
}
__host__ __device__ inline dd operator*(double a, const dd &b) {
    SPHBI_DD_EXACT
    return b * a;
}
__host__ __device__ inline dd operator/(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    const double q1 = a.hi / b.hi;
    dd r = a - b * q1;
    const double q2 = r.hi / b.hi;
    r = r - b * q2;
    const double q3 = r.hi / b.hi;
    return fast_two_sum(q1, q2) + q3;
}
__host__ __device__ inline dd operator/(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a / dd(b);
}
__host__ __device__ inline dd operator/(double a, const dd &b) {
    SPHBI_DD_EXACT
    return dd(a) / b;
}
__host__ __device__ inline dd &operator+=(dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return a = a + b;
}
__host__ __device__ inline dd &operator-=(dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return a = a - b;
}
__host__ __device__ inline dd &operator*=(dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return a = a * b;
}

// ---- comparisons (by value: hi decides, lo breaks ties)
__host__ __device__ inline bool operator<(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}
__host__ __device__ inline bool operator>(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return b < a;
}
__host__ __device__ inline bool operator<=(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return !(b < a);
}
__host__ __device__ inline bool operator>=(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return !(a < b);
}
__host__ __device__ inline bool operator==(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return a.hi == b.hi && a.lo == b.lo;
}
__host__ __device__ inline bool operator!=(const dd &a, const dd &b) {
    SPHBI_DD_EXACT
    return !(a == b);
}
__host__ __device__ inline bool operator<(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a < dd(b);
}
__host__ __device__ inline bool operator>(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a > dd(b);
}
__host__ __device__ inline bool operator<=(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a <= dd(b);
}
__host__ __device__ inline bool operator>=(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a >= dd(b);
}
__host__ __device__ inline bool operator==(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a == dd(b);
}
__host__ __device__ inline bool operator!=(const dd &a, double b) {
    SPHBI_DD_EXACT
    return a != dd(b);
}

__host__ __device__ inline dd fabs(const dd &a) {
    SPHBI_DD_EXACT
    return a.hi < 0.0 ? -a : a;
}
__host__ __device__ inline dd copysign(const dd &a, const dd &s) {
    SPHBI_DD_EXACT
    return (s.hi < 0.0) != (a.hi < 0.0) ? -a : a;
}
// a b + c with the product left unnormalised: (p, e) goes straight into the
// addition, which only needs |e| small beside p (the error is that of the
// addition, a few units of 2^-106 of |a b| + |c|)
__host__ __device__ inline dd fma(const dd &a, const dd &b, const dd &c) {
    SPHBI_DD_EXACT
    const dd p = two_prod(a.hi, b.hi);
    const double e = ::fma(a.hi, b.lo, ::fma(a.lo, b.hi, p.lo));
    dd s = two_sum(p.hi, c.hi);
    s.lo += e + c.lo;
    return fast_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd fma(double a, const dd &b, const dd &c) {
    SPHBI_DD_EXACT
    const dd p = two_prod(a, b.hi);
    const double e = ::fma(a, b.lo, p.lo);
    dd s = two_sum(p.hi, c.hi);
    s.lo += e + c.lo;
    return fast_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd fma(const dd &a, double b, const dd &c) {
    SPHBI_DD_EXACT
    return fma(b, a, c);
}
__host__ __device__ inline dd ldexp(const dd &a, int e) {
    SPHBI_DD_EXACT
    return dd(::ldexp(a.hi, e), ::ldexp(a.lo, e));
}

}  // namespace ddarith

// 1/n as a double-double: q1 = fl(1/n), and the remainder 1 - q1 n formed
// exactly with TwoProduct (1 - p is exact by Sterbenz's lemma).  For a
// constant n the compiler folds it to two constants.
__host__ __device__ inline dd dd_recip(int n) {
    SPHBI_DD_EXACT
    const double x = (double)n;
    const double q1 = 1.0 / x;
    const dd p = two_prod(q1, x);
    const double r = (1.0 - p.hi) - p.lo;
    return fast_two_sum(q1, r / x);
}

// pi/2 (its two leading 53-bit pieces) and ln 2
__host__ __device__ constexpr dd dd_pi2() {
    SPHBI_DD_EXACT
    return dd(1.570796326794896558, 6.123233995736766e-17);
}
__host__ __device__ constexpr dd dd_ln2() {
    SPHBI_DD_EXACT
    return dd(0.6931471805599452862, 2.3190468138462996e-17);
}

__host__ __device__ inline dd dd_sqrt(const dd &a) {
    SPHBI_DD_EXACT
    if (!(a.hi > 0.0)) return dd(0.0);
    const double x = sqrt(a.hi);
    const dd r = a - two_prod(x, x);
    return fast_two_sum(x, r.hi * (0.5 / x));
}

// log(a) for a > 0: a = m 2^e with m in [1/sqrt 2, sqrt 2); log m = 2 atanh(s),
// s = (m - 1)/(m + 1), |s| <= 0.1716, by its series sum s^(2k+1)/(2k+1) to
// k = 21 (the next term is below 2^-106 relative).
__host__ __device__ inline dd dd_log(const dd &a) {
    SPHBI_DD_EXACT
    int e = 0;
    (void)frexp(a.hi, &e);
    dd m = ldexp(a, -e);                         // [1/2, 1)
    if (m.hi < 0.7071067811865476) {
        m = ldexp(m, 1);
        e -= 1;
    }
    const dd s = (m - 1.0) / (m + 1.0);
    const dd s2 = s * s;
    dd q = dd_recip(43);
#pragma unroll
    for (int k = 20; k >= 0; --k) q = q * s2 + dd_recip(2 * k + 1);
    return ldexp(s * q, 1) + dd_ln2() * (double)e;
}

// atan(y/x) for y >= 0, x > 0.  After swapping to a ratio t <= 1 the
// half-angle identity atan t = 2 atan(t / (1 + sqrt(1 + t^2))) is applied
// three times (t <= tan(pi/32) < 0.0985), then the series
// sum (-1)^k t^(2k+1)/(2k+1) to k = 16.
__host__ __device__ inline dd dd_atan2_q1(const dd &y, const dd &x) {
    SPHBI_DD_EXACT
    const bool swap = y > x;
    dd t = swap ? x / y : y / x;
#pragma unroll
    for (int i = 0; i < 3; ++i) t = t / (1.0 + dd_sqrt(1.0 + t * t));
    const dd t2 = t * t;
    dd q = dd_recip(33);
#pragma unroll
    for (int k = 15; k >= 0; --k) q = dd_recip(2 * k + 1) - q * t2;     // 1 - t^2 (1/3 - t^2 (1/5 - ...))
    const dd a = ldexp(t * q, 3);
    return swap ? dd_pi2() - a : a;
}

// Precision policy of the double-double pairs (the interface of ExactMath in
// precision.h, on double-double arguments).
struct DDMath {
    __host__ __device__ dd sqrt_(const dd &x) const { return dd_sqrt(x); }
    __host__ __device__ dd rsqrt_(const dd &x) const { return 1.0 / dd_sqrt(x); }
    __host__ __device__ dd rcp_(const dd &x) const { return 1.0 / x; }
    __host__ __device__ dd sector_angle(const dd &p, const dd &ay, const dd &yc) const {
        dd num = p * (ay - yc);
        if (num.hi < 0.0) num = dd(0.0);
        return dd_atan2_q1(num, p * p + ay * yc);
    }
    // H_0 = asinh(yB/p) - asinh(yA/p) with asinh(|y|/p) = log((|y| + rho)/p)
    __host__ __device__ dd h0(const dd &p, const dd &yA, const dd &yB, const dd &rA, const dd &rB) const {
        const dd gA = fabs(yA) + rA, gB = fabs(yB) + rB;
        dd num, den;
        double sg;
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
        return dd_log(num / den) * sg;
    }
    __host__ __device__ void edge_norm(const dd &len2, dd &len, dd &il) const {
        len = dd_sqrt(len2);
        il = 1.0 / len;
    }
    __host__ __device__ DDMath for_edge(const dd &, double) const { return *this; }
};

}  // namespace sphbi
