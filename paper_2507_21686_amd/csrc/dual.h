// Forward-mode dual numbers: a value and N directional derivatives.
// Used by the adjoint kernel to differentiate the closed-form pair
// evaluation with respect to the triangle vertices.
#pragma once

#include <math.h>

namespace sphbi {

template <int N>
struct Dual {
    double v;
    double d[N];
    __host__ __device__ Dual() : v(0.0) {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual(double x) : v(x) {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual &operator+=(const Dual &b) {
        v += b.v;
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] += b.d[i];
        return *this;
    }
    __host__ __device__ Dual &operator-=(const Dual &b) {
        v -= b.v;
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] -= b.d[i];
        return *this;
    }
    __host__ __device__ Dual &operator*=(const Dual &b) {
        *this = *this * b;
        return *this;
    }
    __host__ __device__ friend Dual operator+(const Dual &a, const Dual &b) {
        Dual r;
        r.v = a.v + b.v;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
        return r;
    }
    __host__ __device__ friend Dual operator-(const Dual &a, const Dual &b) {
        Dual r;
        r.v = a.v - b.v;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
        return r;
    }
    __host__ __device__ friend Dual operator-(const Dual &a) {
        Dual r;
        r.v = -a.v;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
        return r;
    }
    __host__ __device__ friend Dual operator*(const Dual &a, const Dual &b) {
        Dual r;
        r.v = a.v * b.v;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
        return r;
    }
    __host__ __device__ friend Dual operator/(const Dual &a, const Dual &b) {
        Dual r;
        const double ib = 1.0 / b.v;
        r.v = a.v * ib;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
        return r;
    }
    __host__ __device__ friend Dual operator+(const Dual &a, double b) {
        Dual r = a;
        r.v += b;
        return r;
    }
    __host__ __device__ friend Dual operator+(double a, const Dual &b) { return b + a; }
    __host__ __device__ friend Dual operator-(const Dual &a, double b) {
        Dual r = a;
        r.v -= b;
        return r;
    }
    __host__ __device__ friend Dual operator-(double a, const Dual &b) {
        Dual r = -b;
        r.v += a;
        return r;
    }
    __host__ __device__ friend Dual operator*(const Dual &a, double b) {
        Dual r;
        r.v = a.v * b;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
        return r;
    }
    __host__ __device__ friend Dual operator*(double a, const Dual &b) { return b * a; }
    __host__ __device__ friend Dual operator/(const Dual &a, double b) { return a * (1.0 / b); }
    __host__ __device__ friend Dual operator/(double a, const Dual &b) { return Dual(a) / b; }

    __host__ __device__ friend bool operator<(const Dual &a, const Dual &b) { return a.v < b.v; }
    __host__ __device__ friend bool operator>(const Dual &a, const Dual &b) { return a.v > b.v; }
    __host__ __device__ friend bool operator<(const Dual &a, double b) { return a.v < b; }
    __host__ __device__ friend bool operator>(const Dual &a, double b) { return a.v > b; }
    __host__ __device__ friend bool operator<=(const Dual &a, double b) { return a.v <= b; }
    __host__ __device__ friend bool operator>=(const Dual &a, double b) { return a.v >= b; }
    __host__ __device__ friend bool operator==(const Dual &a, double b) { return a.v == b; }
    __host__ __device__ friend bool operator!=(const Dual &a, double b) { return a.v != b; }
    __host__ __device__ friend bool operator<(double a, const Dual &b) { return a < b.v; }
    __host__ __device__ friend bool operator>(double a, const Dual &b) { return a > b.v; }

    __host__ __device__ friend Dual sqrt(const Dual &a) {
        Dual r;
        r.v = ::sqrt(a.v);
        const double f = r.v > 0.0 ? 0.5 / r.v : 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * f;
        return r;
    }
    __host__ __device__ friend Dual log(const Dual &a) {
        Dual r;
        r.v = ::log(a.v);
        const double f = 1.0 / a.v;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * f;
        return r;
    }
    __host__ __device__ friend Dual fabs(const Dual &a) { return a.v < 0.0 ? -a : a; }
    __host__ __device__ friend Dual copysign(const Dual &a, const Dual &b) {
        const bool flip = (a.v < 0.0) != (b.v < 0.0);
        return flip ? -a : a;
    }
    __host__ __device__ friend Dual atan2(const Dual &y, const Dual &x) {
        Dual r;
        r.v = ::atan2(y.v, x.v);
        const double den = x.v * x.v + y.v * y.v;
        const double f = den > 0.0 ? 1.0 / den : 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) * f;
        return r;
    }
    __host__ __device__ friend Dual fma(const Dual &a, const Dual &b, const Dual &c) { return a * b + c; }
    __host__ __device__ friend Dual fma(double a, const Dual &b, const Dual &c) { return b * a + c; }
};

}  // namespace sphbi
