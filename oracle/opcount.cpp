/*
 * oracle/opcount.cpp -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY.
 *
 * The closed-form oracle (closed_form.c: the decomposition of Sec. 4 and the
 * closed forms of Sec. 5) compiled with an operation-counting scalar in place
 * of double.  Every floating-point operation with a counted operand is
 * tallied by kind: additions and subtractions, multiplications, divisions,
 * square roots and transcendental calls (log, atan2, cos, sin).  Operations
 * between plain constants (table indices, loop bounds) stay uncounted, as a
 * compiler folds them.  The counts of one pair are the algorithmic work of
 * the paper's method for that pair; the measurement tools divide the
 * device's measured rate into them.  Only measurement scripts and tests load
 * this library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

namespace {

enum { C_ADD, C_MUL, C_DIV, C_SQRT, C_TRANS, C_N };
thread_local long long g_count[C_N];

struct cnt_t {
    double v;
    cnt_t() = default;
    cnt_t(double x) : v(x) {}
    cnt_t(int x) : v(x) {}
    explicit operator double() const { return v; }
};
static_assert(sizeof(cnt_t) == sizeof(double), "layout of double");

inline cnt_t op(int kind, double r) { ++g_count[kind]; return cnt_t(r); }

inline cnt_t operator+(cnt_t a, cnt_t b) { return op(C_ADD, a.v + b.v); }
inline cnt_t operator-(cnt_t a, cnt_t b) { return op(C_ADD, a.v - b.v); }
inline cnt_t operator*(cnt_t a, cnt_t b) { return op(C_MUL, a.v * b.v); }
inline cnt_t operator/(cnt_t a, cnt_t b) { return op(C_DIV, a.v / b.v); }
inline cnt_t operator+(cnt_t a, double b) { return op(C_ADD, a.v + b); }
inline cnt_t operator-(cnt_t a, double b) { return op(C_ADD, a.v - b); }
inline cnt_t operator*(cnt_t a, double b) { return op(C_MUL, a.v * b); }
inline cnt_t operator/(cnt_t a, double b) { return op(C_DIV, a.v / b); }
inline cnt_t operator+(double a, cnt_t b) { return op(C_ADD, a + b.v); }
inline cnt_t operator-(double a, cnt_t b) { return op(C_ADD, a - b.v); }
inline cnt_t operator*(double a, cnt_t b) { return op(C_MUL, a * b.v); }
inline cnt_t operator/(double a, cnt_t b) { return op(C_DIV, a / b.v); }
inline cnt_t operator-(cnt_t a) { return cnt_t(-a.v); }
inline cnt_t &operator+=(cnt_t &a, cnt_t b) { return a = a + b; }
inline cnt_t &operator-=(cnt_t &a, cnt_t b) { return a = a - b; }
inline cnt_t &operator*=(cnt_t &a, cnt_t b) { return a = a * b; }
inline cnt_t &operator/=(cnt_t &a, cnt_t b) { return a = a / b; }
inline bool operator<(cnt_t a, cnt_t b) { return a.v < b.v; }
inline bool operator>(cnt_t a, cnt_t b) { return a.v > b.v; }
inline bool operator<=(cnt_t a, cnt_t b) { return a.v <= b.v; }
inline bool operator>=(cnt_t a, cnt_t b) { return a.v >= b.v; }
inline bool operator==(cnt_t a, cnt_t b) { return a.v == b.v; }
inline bool operator!=(cnt_t a, cnt_t b) { return a.v != b.v; }
inline bool operator!(cnt_t a) { return !a.v; }

inline cnt_t sqrt(cnt_t a) { return op(C_SQRT, ::sqrt(a.v)); }
inline cnt_t log(cnt_t a) { return op(C_TRANS, ::log(a.v)); }
inline cnt_t cos(cnt_t a) { return op(C_TRANS, ::cos(a.v)); }
inline cnt_t sin(cnt_t a) { return op(C_TRANS, ::sin(a.v)); }
inline cnt_t atan2(cnt_t a, cnt_t b) { return op(C_TRANS, ::atan2(a.v, b.v)); }
inline cnt_t fabs(cnt_t a) { return cnt_t(::fabs(a.v)); }
inline cnt_t fmax(cnt_t a, cnt_t b) { return cnt_t(::fmax(a.v, b.v)); }
inline cnt_t fmin(cnt_t a, cnt_t b) { return cnt_t(::fmin(a.v, b.v)); }
inline bool cnt_isfinite(cnt_t a) { return ::isfinite(a.v); }

}  // namespace

#undef isfinite
#define isfinite cnt_isfinite
#define double cnt_t
#define oracle_cf_radial opcount_cf_radial
#define oracle_cf_pair opcount_cf_pair
#define oracle_cf_integrate opcount_cf_integrate
// the kernel monomials come from definition.c (C linkage; cnt_t has the
// layout of double)
extern "C" int oracle_kernel_monomials(int id, int *npieces, cnt_t *R, int *deg, cnt_t *b, cnt_t *Cd);
#include "closed_form.c"
#undef double
#undef isfinite

/* Operation counts of one pair in the support-normalised frame (particle at
 * the origin, support 1): counts[0..4] = additions, multiplications,
 * divisions, square roots, transcendental calls; out = (I, Gx, Gy) of the
 * counted evaluation (identical to the closed-form oracle's); cls = number
 * of vertices inside the support (the case of Sec. 4.6).  Returns 0. */
extern "C" int oracle_opcount_pair(int kid, int nn, const double *tri6, const double *A, double *out,
                                   long long *counts, int *cls) {
    cnt_t v[3][2], a[10], o[3];
    for (int i = 0; i < 3; ++i) {
        v[i][0] = cnt_t(tri6[2 * i]);
        v[i][1] = cnt_t(tri6[2 * i + 1]);
    }
    for (int i = 0; i < nn && i < 10; ++i) a[i] = cnt_t(A[i]);
    int ni = 0;
    for (int i = 0; i < 3; ++i) ni += tri6[2 * i] * tri6[2 * i] + tri6[2 * i + 1] * tri6[2 * i + 1] <= 1.0;
    *cls = ni;
    memset(g_count, 0, sizeof(g_count));
    cf_pair_normalised(kid, nn, v, a, o);
    for (int k = 0; k < C_N; ++k) counts[k] = g_count[k];
    for (int k = 0; k < 3; ++k) out[k] = (double)o[k];
    return 0;
}
