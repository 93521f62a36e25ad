// Closed-form pair mathematics shared by the forward and adjoint kernels.
// The scalar type S is double, or the double-double type of ddmath.h for the
// ill-conditioned pairs; the precision policy M decides how the square
// roots, reciprocals, angles and logarithms are evaluated, and the kernel
// description K (KArgs, or KArgsDD for double-double) supplies the kernel's
// coefficients.  See forward_pair.h for the derivation.
#pragma once

#include <math.h>

#include "ddmath.h"
#include "internal.h"
#include "precision.h"

namespace sphbi {

__host__ __device__ constexpr int pidx(int i, int j) { return (i + j) * (i + j + 1) / 2 + j; }

// An FP64 constant as an instruction operand: the values the hardware encodes
// inline (0, +-1/2, +-1, +-2, +-4) stay literal, every other one is handed
// over through a scalar register at its point of use (see sconst()).  Only a
// value the compiler knows at compile time (after inlining and unrolling)
// takes the scalar-register path; any other value is returned as it is, so
// a lane-varying value can never be forced into a scalar register.
__device__ inline double lit(double c) {
    if (!__builtin_constant_p(c)) return c;
    const double a = fabs(c);
    return (a == 0.0 || a == 0.5 || a == 1.0 || a == 2.0 || a == 4.0) ? c : sconst(c);
}

// 1/n for a small integer n in the scalar type of a pair: an FP64 constant
// handed over like lit(), or the double-double nearest to 1/n.
template <typename S>
struct RecipInt {
    __device__ static double get(int n) { return lit(1.0 / n); }
};
template <>
struct RecipInt<dd> {
    __host__ __device__ static dd get(int n) { return dd_recip(n); }
};

// The kernel coefficients of a piece, for field degree m (see KArgs):
// b_k / (k + 2 + m), k b_k / (k + 1 + m) and the unit-sector integrals.
__device__ inline double coef_bq(const KArgs &K, int pc, int m, int k) { return K.bq[pc][m][k]; }
__device__ inline double coef_kbq(const KArgs &K, int pc, int m, int k) { return K.kbq[pc][m][k]; }
__device__ inline double coef_sv(const KArgs &K, int pc, int m) { return K.sv[pc][m]; }
__device__ inline double coef_sw(const KArgs &K, int pc, int m) { return K.sw[pc][m]; }

// Double-double kernel description: the monomial coefficients b exactly as
// given, the quotients formed in double-double where they are used, the
// unit-sector integrals in double-double (made on the host by
// make_kargs_dd).
struct KArgsDD {
    int npieces;
    int pad;
    double R[2];
    double iR[2];
    double b[2][kMaxDeg + 1];
    dd sv[2][kMaxOrder + 1];
    dd sw[2][kMaxOrder + 1];
    double cd;
};
__host__ __device__ inline dd coef_bq(const KArgsDD &K, int pc, int m, int k) {
    return K.b[pc][k] * dd_recip(k + 2 + m);
}
__host__ __device__ inline dd coef_kbq(const KArgsDD &K, int pc, int m, int k) {
    return (K.b[pc][k] * (double)k) * dd_recip(k + 1 + m);
}
__host__ __device__ inline dd coef_sv(const KArgsDD &K, int pc, int m) { return K.sv[pc][m]; }
__host__ __device__ inline dd coef_sw(const KArgsDD &K, int pc, int m) { return K.sw[pc][m]; }

// Chebyshev coefficients: T_n(x) = sum_j chebT(n,j) x^j, U_n likewise.
__host__ __device__ constexpr double chebT(int n, int j) {
    return n == 0 ? (j == 0 ? 1.0 : 0.0)
         : n == 1 ? (j == 1 ? 1.0 : 0.0)
         : n == 2 ? (j == 0 ? -1.0 : j == 2 ? 2.0 : 0.0)
         : n == 3 ? (j == 1 ? -3.0 : j == 3 ? 4.0 : 0.0)
         : n == 4 ? (j == 0 ? 1.0 : j == 2 ? -8.0 : j == 4 ? 8.0 : 0.0)
                  : 0.0;
}
__host__ __device__ constexpr double chebU(int n, int j) {
    return n == 0 ? (j == 0 ? 1.0 : 0.0)
         : n == 1 ? (j == 1 ? 2.0 : 0.0)
         : n == 2 ? (j == 0 ? -1.0 : j == 2 ? 4.0 : 0.0)
         : n == 3 ? (j == 1 ? -4.0 : j == 3 ? 8.0 : 0.0)
                  : 0.0;
}

// ----------------------------------------------------------------------------
// field preparation: nodal values -> polynomial about vertex 0 (units of h)
// ----------------------------------------------------------------------------
template <typename S>
__host__ __device__ inline void mul_affine(const S *in, S a, S bx, S by, S *out) {
#pragma unroll
    for (int m = 0; m <= 3; ++m)
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            const int i = m - j;
            S v = a * in[pidx(i, j)];
            if (i > 0) v += bx * in[pidx(i - 1, j)];
            if (j > 0) v += by * in[pidx(i, j - 1)];
            out[pidx(i, j)] = v;
        }
}

// Lagrange basis of the element as polynomials in eta = (x - v0)/h: calls
// fn(node, weight, t) for every node, where weight * t (t ordered like the
// record's field coefficients) is the node's basis function.  Nothing is
// called for a degenerate triangle.
template <int ORDER, typename S, typename F>
__host__ __device__ inline void for_each_basis(const S *v, double invh, F &&fn) {
    if (ORDER == 0) {
        S t[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) t[k] = k == 0 ? 1.0 : 0.0;
        fn(0, 1.0, t);
        return;
    }
    const S q1x = (v[2] - v[0]) * invh, q1y = (v[3] - v[1]) * invh;
    const S q2x = (v[4] - v[0]) * invh, q2y = (v[5] - v[1]) * invh;
    const S det = q1x * q2y - q1y * q2x;
    if (det == 0.0) return;
    const S id = 1.0 / det;
    // barycentric coordinates as affine forms in eta (origin at v0)
    const S l1x = q2y * id, l1y = -q2x * id;
    const S l2x = -q1y * id, l2y = q1x * id;
    const S la[3] = {1.0, 0.0, 0.0};
    const S lx[3] = {-(l1x + l2x), l1x, l2x};
    const S ly[3] = {-(l1y + l2y), l1y, l2y};
    S one[10], t1[10], t2[10], t3[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) one[k] = k == 0 ? 1.0 : 0.0;
    if (ORDER == 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mul_affine(one, la[i], lx[i], ly[i], t1);
            fn(i, 1.0, t1);
        }
        return;
    }
    // vertices: lambda (3 lambda - 1)(3 lambda - 2) / 2
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        mul_affine(one, la[i], lx[i], ly[i], t1);
        mul_affine(t1, 3.0 * la[i] - 1.0, 3.0 * lx[i], 3.0 * ly[i], t2);
        mul_affine(t2, 3.0 * la[i] - 2.0, 3.0 * lx[i], 3.0 * ly[i], t3);
        fn(i, 0.5, t3);
    }
    // edge nodes: 9/2 lambda_a lambda_b (3 lambda_a - 1) at 1/3 from a,
    //             9/2 lambda_a lambda_b (3 lambda_b - 1) at 2/3 from a
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
        const int a = ed, b = (ed + 1) % 3;
        mul_affine(one, la[a], lx[a], ly[a], t1);
        mul_affine(t1, la[b], lx[b], ly[b], t2);
        mul_affine(t2, 3.0 * la[a] - 1.0, 3.0 * lx[a], 3.0 * ly[a], t3);
        fn(3 + 2 * ed, 4.5, t3);
        mul_affine(t2, 3.0 * la[b] - 1.0, 3.0 * lx[b], 3.0 * ly[b], t3);
        fn(4 + 2 * ed, 4.5, t3);
    }
    // centroid: 27 lambda_0 lambda_1 lambda_2
    mul_affine(one, la[0], lx[0], ly[0], t1);
    mul_affine(t1, la[1], lx[1], ly[1], t2);
    mul_affine(t2, la[2], lx[2], ly[2], t3);
    fn(9, 27.0, t3);
}

// One record: vertices v[6] (world units) and nodal values A[n_nodes] ->
// rec[16] = v, then e_ij of A(v0 + h eta) = sum e_ij eta_x^i eta_y^j.
template <int ORDER, typename S>
__host__ __device__ inline void prepare_record(const S *v, const S *A, double invh, S *r) {
    S e[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) e[k] = 0.0;
    for_each_basis<ORDER, S>(v, invh, [&](int i, double w, const S *t) {
#pragma unroll
        for (int k = 0; k < 10; ++k) e[k] += w * A[i] * t[k];
    });
#pragma unroll
    for (int k = 0; k < 6; ++k) r[k] = v[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) r[6 + k] = e[k];
}

// Transpose of the field preparation: for weights g on the coefficients e_ij,
// gA[i] = sum_ij g_ij d e_ij / d A_i (the basis function's coefficients
// dotted with g).
template <int ORDER, typename S>
__host__ __device__ inline void prepare_record_T(const S *v, const S *g, double invh, S *gA) {
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
#pragma unroll
    for (int i = 0; i < NN; ++i) gA[i] = 0.0;
    for_each_basis<ORDER, S>(v, invh, [&](int i, double w, const S *t) {
        S d = 0.0;
#pragma unroll
        for (int k = 0; k < 10; ++k) d += t[k] * g[k];
#pragma unroll
        for (int n = 0; n < NN; ++n)
            if (n == i) gA[n] = w * d;
    });
}

// ----------------------------------------------------------------------------
// per-pair closed form
// ----------------------------------------------------------------------------

// Harmonics of a degree-m homogeneous part: A_m(psi) = sum_n hc[n] cos(n psi) + hs[n] sin(n psi)
template <typename S>
struct Harm {
    S c[5], s[5];
};

// A_m(psi) * cos(psi) and A_m(psi) * sin(psi) (product-to-sum)
template <typename S>
__host__ __device__ inline void mul_cs(int M, const Harm<S> &v, Harm<S> &x, Harm<S> &y) {
#pragma unroll
    for (int n = 0; n < 5; ++n) { x.c[n] = x.s[n] = y.c[n] = y.s[n] = 0.0; }
#pragma unroll
    for (int n = M & 1; n <= M; n += 2) {
        const S c = v.c[n], s = v.s[n];
        if (n == 0) {
            x.c[1] += c;
            y.s[1] += c;
        } else {
            x.c[n + 1] += 0.5 * c;
            x.c[n - 1] += 0.5 * c;
            x.s[n + 1] += 0.5 * s;
            if (n - 1 > 0) x.s[n - 1] += 0.5 * s;
            y.s[n + 1] += 0.5 * c;
            if (n - 1 > 0) y.s[n - 1] -= 0.5 * c;
            y.c[n - 1] += 0.5 * s;
            y.c[n + 1] -= 0.5 * s;
        }
    }
}

// Transpose of mul_cs: weights x, y on the harmonics of A_m cos(psi) and
// A_m sin(psi) -> weights added to the harmonic slots of A_m.
template <typename S>
__host__ __device__ inline void mul_cs_T(int M, const Harm<S> &x, const Harm<S> &y, Harm<S> &d) {
#pragma unroll
    for (int n = M & 1; n <= M; n += 2) {
        if (n == 0) {
            d.c[0] += x.c[1] + y.s[1];
        } else {
            const S ys = n > 1 ? y.s[n - 1] : S(0.0), xs = n > 1 ? x.s[n - 1] : S(0.0);
            d.c[n] += 0.5 * (x.c[n + 1] + x.c[n - 1] + y.s[n + 1] - ys);
            d.s[n] += 0.5 * (x.s[n + 1] + xs + y.c[n - 1] - y.c[n + 1]);
        }
    }
}

template <int ORDER, typename S>
__host__ __device__ inline void global_harmonics(const S *c, Harm<S> *h) {
#pragma unroll
    for (int m = 0; m <= ORDER; ++m)
#pragma unroll
        for (int n = 0; n < 5; ++n) h[m].c[n] = h[m].s[n] = 0.0;
    h[0].c[0] = c[0];
    if (ORDER >= 1) {
        h[1].c[1] = c[pidx(1, 0)];
        h[1].s[1] = c[pidx(0, 1)];
    }
    if (ORDER >= 2) {
        const S c20 = c[pidx(2, 0)], c11 = c[pidx(1, 1)], c02 = c[pidx(0, 2)];
        h[2].c[0] = 0.5 * (c20 + c02);
        h[2].c[2] = 0.5 * (c20 - c02);
        h[2].s[2] = 0.5 * c11;
    }
    if (ORDER >= 3) {
        const S c30 = c[pidx(3, 0)], c21 = c[pidx(2, 1)], c12 = c[pidx(1, 2)], c03 = c[pidx(0, 3)];
        h[3].c[1] = lit(0.25) * fma(lit(3.0), c30, c12);
        h[3].s[1] = lit(0.25) * fma(lit(3.0), c03, c21);
        h[3].c[3] = lit(0.25) * (c30 - c12);
        h[3].s[3] = lit(0.25) * (c21 - c03);
    }
}

// A(xi) = sum e_ij (xi - s)^(i,j): coefficients about the particle
template <int ORDER, typename S>
__host__ __device__ inline void taylor_shift(const S *__restrict__ e, S sx, S sy, S *c) {
    // powers of -s
    const S mx[4] = {1.0, -sx, sx * sx, -sx * sx * sx};
    const S my[4] = {1.0, -sy, sy * sy, -sy * sy * sy};
    constexpr double B[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
#pragma unroll
    for (int k = 0; k < 10; ++k) c[k] = 0.0;
#pragma unroll
    for (int mi = 0; mi <= ORDER; ++mi)
#pragma unroll
        for (int j = 0; j <= mi; ++j) {
            const int i = mi - j;
            const S eij = e[pidx(i, j)];
#pragma unroll
            for (int a = 0; a <= i; ++a)
#pragma unroll
                for (int b = 0; b <= j; ++b) {
                    const double w = B[i][a] * B[j][b];
                    const S f = w == 1.0 ? eij : S(eij * lit(w));
                    c[pidx(a, b)] += f * mx[i - a] * my[j - b];
                }
        }
}

// Consumers of the per-edge closed forms.  edge_piece() hands each one the
// edge-frame integrals of every harmonic slot: the sector parts (angular
// terms times the unit-sector radial integrals sv, sw) and the triangle parts
// (value harmonics n = m, m-2, ... and gradient harmonics n = m+1, m-1, ...
// of the degree-m part of the field).
//
// A sink may also take the radial terms themselves (radial(), after they are
// formed): kHMax, kPMax are the largest indices of H and P it reads beyond the
// contraction's, and kOnLine says the edge may lie on a line through the
// particle (p = 0), where H_0 is taken as 0 (it only ever appears times p).
//
// FieldSink contracts them with the edge-frame harmonics hv of NF fields and
// adds each field's value and gradient integrals (without c_d and the -1/h of
// the gradient).
template <typename S, int NF = 1>
struct FieldSink {
    static constexpr int kHMax = 0, kPMax = 0;
    static constexpr bool kOnLine = false;
    template <typename KA>
    __host__ __device__ void radial(const KA &, int, S, const S *, const S *) {}
    const Harm<S> *hv[NF];          // NF fields sharing the geometry
    S I[NF], X[NF], Y[NF];
    Harm<S> hx[NF], hy[NF];
    template <typename C>
    __host__ __device__ void sector(int m, C sv, C sw, const S *angc, const S *angs) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Harm<S> gx, gy;
            mul_cs(m, hv[f][m], gx, gy);
#pragma unroll
            for (int n = m & 1; n <= m; n += 2) I[f] += sv * (hv[f][m].c[n] * angc[n] + hv[f][m].s[n] * angs[n]);
#pragma unroll
            for (int n = (m + 1) & 1; n <= m + 1; n += 2) {
                X[f] += sw * (gx.c[n] * angc[n] + gx.s[n] * angs[n]);
                Y[f] += sw * (gy.c[n] * angc[n] + gy.s[n] * angs[n]);
            }
        }
    }
    __host__ __device__ void begin(int m) {
#pragma unroll
        for (int f = 0; f < NF; ++f) mul_cs(m, hv[f][m], hx[f], hy[f]);
    }
    __host__ __device__ void value(int m, int n, S vc, S vs) {
#pragma unroll
        for (int f = 0; f < NF; ++f) I[f] += hv[f][m].c[n] * vc + hv[f][m].s[n] * vs;
    }
    __host__ __device__ void grad(int, int n, S wc, S ws) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            X[f] += hx[f].c[n] * wc + hx[f].s[n] * ws;
            Y[f] += hy[f].c[n] * wc + hy[f].s[n] * ws;
        }
    }
};

// BasisSink keeps the integrals themselves, summed over the kernel pieces:
// vb[m] for the value slots and gb[m] for the gradient slots.  Every
// quantity of the pair that is linear in the field is a dot product of these
// with the field's harmonics (the adjoint uses this to get the moments of all
// monomials at the cost of one evaluation).
template <int ORDER, typename S>
struct BasisSink {
    static constexpr int kHMax = 0, kPMax = 0;
    static constexpr bool kOnLine = false;
    template <typename KA>
    __host__ __device__ void radial(const KA &, int, S, const S *, const S *) {}
    Harm<S> vb[ORDER + 1], gb[ORDER + 1];
    template <typename C>
    __host__ __device__ void sector(int m, C sv, C sw, const S *angc, const S *angs) {
#pragma unroll
        for (int n = m & 1; n <= m; n += 2) {
            vb[m].c[n] += sv * angc[n];
            vb[m].s[n] += sv * angs[n];
        }
#pragma unroll
        for (int n = (m + 1) & 1; n <= m + 1; n += 2) {
            gb[m].c[n] += sw * angc[n];
            gb[m].s[n] += sw * angs[n];
        }
    }
    __host__ __device__ void begin(int) {}
    __host__ __device__ void value(int m, int n, S vc, S vs) {
        vb[m].c[n] += vc;
        vb[m].s[n] += vs;
    }
    __host__ __device__ void grad(int m, int n, S wc, S ws) {
        gb[m].c[n] += wc;
        gb[m].s[n] += ws;
    }
};

// Boundary line integrals of the adjoint: the transport term of an edge that
// moves with its vertices.  For the edge from a to b, t = (y - ya)/(yb - ya),
//   Ja = int (1 - t) A Phi ds,   Jb = int t A Phi ds,
// Phi = cI W + cX dW/dx_p + cY dW/dy_p, taken over the part of the edge inside
// the support.  On the edge line (distance p, coordinate y, rho^2 = p^2 + y^2)
// the integrand is a polynomial in y times W(rho) or W'(rho)/rho, and with
// y^a = y^(a mod 2) (rho^2 - p^2)^(a div 2) every term reduces to the radial
// terms of edge_piece, H_c = int rho^(c-1) dy and P_e = int y rho^(e-1) dy.
// add() folds in the kernel piece by piece (the pieces share p):
//   G0[i] = sum_j b_j H_(2i+j+1),    G1[i] = sum_j b_j P_(2i+j+1),
//   K0[i] = sum_j j b_j H_(2i+j-1),  K1[i] = sum_j j b_j P_(2i+j-1),
// and finish() expands, with m = a div 2,
//   int y^a W dy              = sum_i C(m,i) (-p^2)^(m-i) (a even ? G0 : G1)[i],
//   h int y^a W'(rho)/rho dy  = the same with K0, K1,
// and contracts them with the field along the line.
template <int DEG, int ORDER, typename S>
struct LineSums {
    static constexpr int NP = ORDER + 2;          // t A has degree ORDER + 1
    static constexpr int NQ = ORDER + 3;          // t A (p gn + y gt) has degree ORDER + 2
    static constexpr int NG0 = (NP + 1) / 2, NG1 = NP / 2, NK0 = (NQ + 1) / 2, NK1 = NQ / 2;
    static constexpr int kHMax = DEG + 2 * NG0 - 1 > DEG + 2 * NK0 - 3 ? DEG + 2 * NG0 - 1 : DEG + 2 * NK0 - 3;
    static constexpr int kPMax = DEG + 2 * NG1 - 1 > DEG + 2 * NK1 - 3 ? DEG + 2 * NG1 - 1 : DEG + 2 * NK1 - 3;
    S G0[NG0], G1[NG1], K0[NK0], K1[NK1];
    __device__ void clear() {
#pragma unroll
        for (int i = 0; i < NG0; ++i) G0[i] = 0.0;
#pragma unroll
        for (int i = 0; i < NG1; ++i) G1[i] = 0.0;
#pragma unroll
        for (int i = 0; i < NK0; ++i) K0[i] = 0.0;
#pragma unroll
        for (int i = 0; i < NK1; ++i) K1[i] = 0.0;
    }
    // the radial terms of piece pc, from ya to yb (either direction)
    template <typename KA>
    __device__ void add(const KA &K, int pc, const S *H, const S *P) {
#pragma unroll
        for (int j = 0; j <= DEG; ++j) {
            if (CoefZeros<KA>::mask >> j & 1u) continue;
            const double bj = K.b[pc][j];
#pragma unroll
            for (int i = 0; i < NG0; ++i) G0[i] = fma(bj, H[2 * i + j + 1], G0[i]);
#pragma unroll
            for (int i = 0; i < NG1; ++i) G1[i] = fma(bj, P[2 * i + j + 1], G1[i]);
            if (j >= 1) {
                const double kb = lit(j) * bj;
#pragma unroll
                for (int i = 0; i < NK0; ++i) K0[i] = fma(kb, H[2 * i + j - 1], K0[i]);
#pragma unroll
                for (int i = 0; i < NK1; ++i) K1[i] = fma(kb, P[2 * i + j - 1], K1[i]);
            }
        }
    }
    // Ja, Jb (world units, c_d and the 1/h of the gradient included) for the
    // edge from ya to yb on the line p n + y tau, tau = (-ny, nx); c is the
    // field about the particle in units of h, record order
    __device__ void finish(S p, S ya, S yb, S nx, S ny, const S *c, double cI, double cX, double cY, double invh,
                           double cd, S &Ja, S &Jb) const {
        // A along the line: xi_x = p nx - y ny, xi_y = p ny + y nx
        S X[ORDER + 1][ORDER + 1], Y[ORDER + 1][ORDER + 1];     // coefficients of xi_x^i, xi_y^i in y
#pragma unroll
        for (int i = 0; i <= ORDER; ++i)
#pragma unroll
            for (int q = 0; q <= ORDER; ++q) X[i][q] = Y[i][q] = 0.0;
        X[0][0] = Y[0][0] = 1.0;
#pragma unroll
        for (int i = 1; i <= ORDER; ++i)
#pragma unroll
            for (int q = 0; q <= i; ++q) {
                X[i][q] = p * nx * X[i - 1][q] + (q > 0 ? S(-ny * X[i - 1][q - 1]) : S(0.0));
                Y[i][q] = p * ny * Y[i - 1][q] + (q > 0 ? S(nx * Y[i - 1][q - 1]) : S(0.0));
            }
        S Ay[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) Ay[q] = 0.0;
#pragma unroll
        for (int m = 0; m <= ORDER; ++m)
#pragma unroll
            for (int j = 0; j <= m; ++j) {
                const int i = m - j;
                const S cij = c[pidx(i, j)];
#pragma unroll
                for (int qa = 0; qa <= i; ++qa)
#pragma unroll
                    for (int qb = 0; qb <= j; ++qb) Ay[qa + qb] += cij * X[i][qa] * Y[j][qb];
            }
        // Pb = t A, Pa = A - Pb
        const S il = 1.0 / (yb - ya);
        S Pa[NP], Pb[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const S prev = q > 0 ? Ay[q - 1] : S(0.0);
            Pb[q] = il * (prev - ya * Ay[q]);
            Pa[q] = Ay[q] - Pb[q];
        }
        // int y^a W dy (U) and h int y^a W'/rho dy (V)
        const S p2 = p * p;
        auto expand = [&](int a, const S *g0, const S *g1) -> S {
            const int m = a >> 1;
            S s = 0.0, pw = 1.0;
#pragma unroll
            for (int i = 2; i >= 0; --i) {
                if (i > m) continue;
                const S gi = (a & 1) ? g1[i] : g0[i];
                const double w = (m == 2 && i == 1) ? 2.0 : 1.0;     // C(m, i), m <= 2
                s = fma(w == 1.0 ? pw : S(lit(w) * pw), gi, s);
                pw *= -p2;
            }
            return s;
        };
        S s1a = 0.0, s1b = 0.0, s2a = 0.0, s2b = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            const S u = expand(a, G0, G1);
            s1a = fma(Pa[a], u, s1a);
            s1b = fma(Pb[a], u, s1b);
        }
        // cX xi_x + cY xi_y = p gn + y gt along the line
        const S gn = cX * nx + cY * ny, gt = cY * nx - cX * ny;
        const S pg = p * gn;
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
            const S v = expand(a, K0, K1);
            S qa = a < NP ? S(pg * Pa[a]) : S(0.0), qb = a < NP ? S(pg * Pb[a]) : S(0.0);
            if (a > 0) {
                qa = fma(gt, Pa[a - 1], qa);
                qb = fma(gt, Pb[a - 1], qb);
            }
            s2a = fma(qa, v, s2a);
            s2b = fma(qb, v, s2b);
        }
        // the radial terms ran from ya to yb
        const S f = yb > ya ? S(cd * invh) : S(-cd * invh);
        Ja = f * (cI * s1a - invh * s2a);
        Jb = f * (cI * s1b - invh * s2b);
    }
};

// BasisSink that also collects the line sums of the same edge.
template <int DEG, int ORDER, typename S>
struct BasisLineSink : BasisSink<ORDER, S> {
    static constexpr int kHMax = LineSums<DEG, ORDER, S>::kHMax, kPMax = LineSums<DEG, ORDER, S>::kPMax;
    LineSums<DEG, ORDER, S> ln;
    template <typename KA>
    __device__ void radial(const KA &K, int pc, S, const S *H, const S *P) { ln.add(K, pc, H, P); }
};

// The line sums alone, for an edge on a line through the particle: it has no
// fan triangle, but its line integral remains.
template <int DEG, int ORDER, typename S>
struct LineSink {
    static constexpr int kHMax = LineSums<DEG, ORDER, S>::kHMax, kPMax = LineSums<DEG, ORDER, S>::kPMax;
    static constexpr bool kOnLine = true;
    LineSums<DEG, ORDER, S> ln;
    template <typename KA>
    __device__ void radial(const KA &K, int pc, S, const S *H, const S *P) { ln.add(K, pc, H, P); }
    template <typename C>
    __device__ void sector(int, C, C, const S *, const S *) {}
    __device__ void begin(int) {}
    __device__ void value(int, int, S, S) {}
    __device__ void grad(int, int, S, S) {}
};

// One edge of the signed fan, one kernel piece of radius R, handed to a sink.
// ra2, rb2 are the squared distances of the edge's ends from the particle: an
// end is clipped (outside the circle) by the same test in both edges that
// share it, which the sector terms below rely on.
template <int DEG, int ORDER, typename S, typename KA, typename M, typename Sink>
__host__ __device__ inline void edge_piece(const KA &K, const M &math, int pc, S p, S ya, S yb, S ra2, S rb2,
                                           Sink &sink) {
    constexpr int HMAX = DEG + ORDER + 1 > Sink::kHMax ? DEG + ORDER + 1 : Sink::kHMax;
    constexpr int PMAX = DEG + ORDER > Sink::kPMax ? DEG + ORDER : Sink::kPMax;
    constexpr unsigned kZ = CoefZeros<KA>::mask;       // b_k known to vanish
    const double R = K.R[pc];
    const S yc = p < R ? S(math.sqrt_((R - p) * (R + p))) : S(0.0);
    const S aya = fabs(ya), ayb = fabs(yb);
    const bool clipA = ra2 > R * R, clipB = rb2 > R * R;

    // ---- sector parts of clipped endpoints (cone formulas, Sec. 5.2)
    // angc[n], angs[n]: integrals of cos(n psi), sin(n psi) over the sector
    // angles of both ends, Q(y_b) - Q(y_a).  The sector of an end runs from the
    // circle crossing psi_c to the end's own ray.  For n >= 1 the part at the
    // end's ray depends only on the ray's direction: in the triangle's frame it
    // is +F(theta_v) from the edge that ends at vertex v and -F(theta_v) from
    // the edge that starts there, so it cancels around the triangle and is not
    // formed (pair_core adds it back where an edge is skipped).  What remains
    // is the angle itself (n = 0) and the crossing part, shared by both ends.
    S angc[5], angs[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) angc[n] = angs[n] = 0.0;
    if (clipA || clipB) {
        double wc = 0.0, ws = 0.0;                    // sums of the ends' signs
#pragma unroll
        for (int end = 0; end < 2; ++end) {
            const bool clip = end ? clipB : clipA;
            if (!clip) continue;
            const S y = end ? yb : ya, ay = end ? ayb : aya;
            const double sg = end ? 1.0 : -1.0;          // Q(y_b) - Q(y_a)
            const double sy = y > 0.0 ? sg : -sg;          // odd cosine part
            wc += sy;
            ws += sg;
            angc[0] += sy * math.sector_angle(p, ay, yc);
        }
        const S cpc = p * K.iR[pc], spc = yc * K.iR[pc];    // (cos, sin) psi_c
        S dn1 = 1.0, tn1 = 0.0, dn = cpc, tn = spc;        // cos/sin of n psi_c
#pragma unroll
        for (int n = 1; n <= ORDER + 1; ++n) {
            const auto inv = RecipInt<S>::get(n);
            angc[n] -= tn * (wc * inv);
            angs[n] += dn * (ws * inv);
            const S dn2 = 2.0 * cpc * dn - dn1, tn2 = 2.0 * cpc * tn - tn1;
            dn1 = dn; tn1 = tn; dn = dn2; tn = tn2;
        }
#pragma unroll
        for (int m = 0; m <= ORDER; ++m) sink.sector(m, coef_sv(K, pc, m), coef_sw(K, pc, m), angc, angs);
    }

    // ---- triangle parts: radial 2F1 terms H_c and powers P_e
    const bool tri = p < R && (aya > 0.0 || ayb > 0.0);
    if (!tri) return;
    S H[HMAX + 1], P[PMAX + 1];
    {
        const S yA = clipA ? S(copysign(yc, ya)) : ya;
        const S yB = clipB ? S(copysign(yc, yb)) : yb;
        const S rA = clipA ? S(R) : S(math.sqrt_(p * p + ya * ya));
        const S rB = clipB ? S(R) : S(math.sqrt_(p * p + yb * yb));
        // H_0 = asinh(yB/p) - asinh(yA/p) with a single logarithm
        const S h0 = math.h0(p, yA, yB, rA, rB);
        const S p2 = p * p;
        H[0] = Sink::kOnLine && !(p > 0.0) ? S(0.0) : h0;
        H[1] = yB - yA;
        S gA = 1.0, gB = 1.0;          // rho^{c-1}
#pragma unroll
        for (int c = 2; c <= HMAX; ++c) {
            gA *= rA;
            gB *= rB;
            H[c] = (gB * yB - gA * yA + lit(c - 1.0) * p2 * H[c - 2]) * RecipInt<S>::get(c);
        }
        S qA = rA, qB = rB;            // rho^{e+1}
#pragma unroll
        for (int e = 0; e <= PMAX; ++e) {
            P[e] = (qB - qA) * RecipInt<S>::get(e + 1);
            qA *= rA;
            qB *= rB;
        }
    }
    sink.radial(K, pc, p, H, P);
    if constexpr (Sink::kOnLine) return;
    S pj[ORDER + 3];
    pj[0] = p;                             // p^{j+1}
#pragma unroll
    for (int j = 1; j < ORDER + 3; ++j) pj[j] = pj[j - 1] * p;

#pragma unroll
    for (int m = 0; m <= ORDER; ++m) {
        sink.begin(m);
        // kernel-contracted radial sums
        S Ac[ORDER + 1], As[ORDER + 1], Bc[ORDER + 2], Bs[ORDER + 1];
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 0; k <= DEG; ++k)
                if (!(kZ >> k & 1u)) s = fma(coef_bq(K, pc, m, k), H[k + 1 + m - j], s);
            Ac[j] = s;
        }
#pragma unroll
        for (int j = 0; j < m; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 0; k <= DEG; ++k)
                if (!(kZ >> k & 1u)) s = fma(coef_bq(K, pc, m, k), P[k + m - j], s);
            As[j] = s;
        }
#pragma unroll
        for (int j = 0; j <= m + 1; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 1; k <= DEG; ++k)
                if (!(kZ >> k & 1u)) s = fma(coef_kbq(K, pc, m, k), H[k + m - j], s);
            Bc[j] = s;
        }
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 1; k <= DEG; ++k)
                if (!(kZ >> k & 1u)) s = fma(coef_kbq(K, pc, m, k), P[k + m - 1 - j], s);
            Bs[j] = s;
        }
        // value harmonics n = m, m-2, ...
#pragma unroll
        for (int n = m & 1; n <= m; n += 2) {
            S vc = 0.0, vs = 0.0;
#pragma unroll
            for (int j = 0; j <= n; ++j)
                if (chebT(n, j) != 0.0) vc = fma(lit(chebT(n, j)) * pj[j], Ac[j], vc);
#pragma unroll
            for (int j = 0; j < n; ++j)
                if (chebU(n - 1, j) != 0.0) vs = fma(lit(chebU(n - 1, j)) * pj[j], As[j], vs);
            sink.value(m, n, vc, vs);
        }
        // gradient harmonics n = m+1, m-1, ...
#pragma unroll
        for (int n = (m + 1) & 1; n <= m + 1; n += 2) {
            S wc = 0.0, ws = 0.0;
#pragma unroll
            for (int j = 0; j <= n; ++j)
                if (chebT(n, j) != 0.0) wc = fma(lit(chebT(n, j)) * pj[j], Bc[j], wc);
#pragma unroll
            for (int j = 0; j < n; ++j)
                if (chebU(n - 1, j) != 0.0) ws = fma(lit(chebU(n - 1, j)) * pj[j], Bs[j], ws);
            sink.grad(m, n, wc, ws);
        }
    }
}

// Frame of the fan edge from a to b (particle at the origin, units of h):
// distance p of the edge line, unit normal n towards it, along-edge
// coordinates ya, yb of the ends from the foot of the perpendicular.  False
// for an edge of zero length or a fan triangle of zero area.
template <typename S, typename M>
__host__ __device__ inline bool edge_frame(const M &math, S axa, S aya, S axb, S ayb, S &p, S &nx, S &ny, S &ya,
                                           S &yb) {
    const S Lx = axb - axa, Ly = ayb - aya;
    const S len2 = Lx * Lx + Ly * Ly;
    if (len2 == 0.0) return false;
    S len, il;
    math.edge_norm(len2, len, il);
    const S tx = Lx * il, ty = Ly * il;
    const S sd = axa * ty - aya * tx;        // signed distance of the edge line
    p = fabs(sd);
    if (p == 0.0) return false;
    nx = sd > 0.0 ? ty : S(-ty);
    ny = sd > 0.0 ? S(-tx) : tx;
    ya = -axa * ny + aya * nx;
    yb = sd > 0.0 ? S(ya + len) : S(ya - len);
    return true;
}

// cos(n phi), sin(n phi) for n <= 3, (cos phi, sin phi) = (nx, ny): the edge
// frame is rotated by phi, and a harmonic of order n by n phi.
template <typename S>
__host__ __device__ inline void edge_phases(S nx, S ny, S *cph, S *sph) {
    cph[0] = 1.0; sph[0] = 0.0;
    cph[1] = nx; sph[1] = ny;
#pragma unroll
    for (int n = 2; n <= 3; ++n) {
        cph[n] = 2.0 * nx * cph[n - 1] - cph[n - 2];
        sph[n] = 2.0 * nx * sph[n - 1] - sph[n - 2];
    }
}

// The part of the sector integrals at a vertex ray that edge_piece leaves out
// (it cancels between the two edges sharing a clipped vertex), for a vertex
// whose partner edge was skipped: s * (F(theta) for every harmonic slot n >= 1
// of the value and the gradient integrand, F_c = sin(n theta)/n and
// F_s = -cos(n theta)/n, summed over the pieces that clip the vertex), in the
// triangle's frame.  (vx, vy): vertex relative to the particle, units of h.
template <int ORDER, typename S, typename KA, typename M>
__host__ __device__ inline void vertex_ray_terms(const KA &K, const M &math, const Harm<S> *hg, S vx, S vy, double s,
                                                 S &oI, S &oX, S &oY) {
    const S r2 = vx * vx + vy * vy;
    if (!(r2 > 0.0)) return;
    const S ir = math.rsqrt_(r2);
    const S c1 = vx * ir, s1 = vy * ir;
    S fc[5], fs[5];                                 // sin(n theta)/n, -cos(n theta)/n
    {
        S cn1 = 1.0, sn1 = 0.0, cn = c1, sn = s1;
        fc[0] = fs[0] = 0.0;
#pragma unroll
        for (int n = 1; n <= ORDER + 1; ++n) {
            const auto inv = RecipInt<S>::get(n);
            fc[n] = sn * inv;
            fs[n] = -cn * inv;
            const S cn2 = 2.0 * c1 * cn - cn1, sn2 = 2.0 * c1 * sn - sn1;
            cn1 = cn; sn1 = sn; cn = cn2; sn = sn2;
        }
#pragma unroll
        for (int n = ORDER + 2; n < 5; ++n) fc[n] = fs[n] = 0.0;
    }
    for (int pc = 0; pc < K.npieces; ++pc) {
        if (!(r2 > K.R[pc] * K.R[pc])) continue;
        S vi = 0.0, vxs = 0.0, vys = 0.0;
#pragma unroll
        for (int m = 0; m <= ORDER; ++m) {
            Harm<S> gx, gy;
            mul_cs(m, hg[m], gx, gy);
            S ti = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll
            for (int n = 1; n < 5; ++n) {
                if (n <= m) ti += hg[m].c[n] * fc[n] + hg[m].s[n] * fs[n];
                if (n <= m + 1) {
                    tx += gx.c[n] * fc[n] + gx.s[n] * fs[n];
                    ty += gy.c[n] * fc[n] + gy.s[n] * fs[n];
                }
            }
            vi += coef_sv(K, pc, m) * ti;
            vxs += coef_sw(K, pc, m) * tx;
            vys += coef_sw(K, pc, m) * ty;
        }
        oI += s * vi;
        oX += s * vxs;
        oY += s * vys;
    }
}

// tau: edges whose line passes within tau (units of h) of the particle are
// evaluated with the exact policy (only meaningful for MixedMath).
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL = 3, typename KA>
__host__ __device__ inline void pair_core(const KA &K, const M &math, double tau, const S *ax, const S *ay,
                                          const S &area2, const S *c, double invh, S &oI, S &oX, S &oY);

// One pair: particle (x, y), record r (vertices and field about vertex 0).
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL = 3, typename KA>
__host__ __device__ inline void pair_fwd(const KA &K, const M &math, double tau, S x, S y, double invh,
                                         const S *__restrict__ r, S &oI, S &oX, S &oY) {
    oI = oX = oY = 0.0;
    S ax[3], ay[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ax[i] = (r[2 * i] - x) * invh;
        ay[i] = (r[2 * i + 1] - y) * invh;
    }
    const S area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
    if (area2 == 0.0) return;
    S c[10];
    taylor_shift<ORDER, S>(r + 6, ax[0], ay[0], c);
    pair_core<DEG, ORDER, S, M, EDGE_UNROLL>(K, math, tau, ax, ay, area2, c, invh, oI, oX, oY);
}

// Number of edges whose line meets the circle of radius^2 R2 about the
// particle (vertices relative to the particle), and the rotation that puts
// those edges first: the start edge when there is one, the edge after the far
// one when there are two.
__host__ __device__ inline int near_edges(const double *ax, const double *ay, double R2, int &rot) {
    bool nr[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int f = e == 2 ? 0 : e + 1;
        const double Lx = ax[f] - ax[e], Ly = ay[f] - ay[e];
        const double l2 = Lx * Lx + Ly * Ly, cr = ax[e] * Ly - ay[e] * Lx;
        nr[e] = l2 > 0.0 && cr * cr < R2 * l2;
    }
    const int near = (int)nr[0] + (int)nr[1] + (int)nr[2];
    rot = near == 1 ? (nr[0] ? 0 : (nr[1] ? 1 : 2)) : near == 2 ? (!nr[0] ? 1 : (!nr[1] ? 2 : 0)) : 0;
    return near;
}

// The same with the triangle's vertices taken from rot (0, 1, 2) on: the
// integrals do not depend on where the edge loop starts, and a common start
// lets the lanes of a wavefront take the same branches (see the sorted
// forward kernel).
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL = 3, typename KA>
__host__ __device__ inline void pair_fwd_rot(const KA &K, const M &math, double tau, S x, S y, double invh,
                                             const S *__restrict__ r, int rot, S &oI, S &oX, S &oY) {
    oI = oX = oY = 0.0;
    S ax[3], ay[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ax[i] = (r[2 * i] - x) * invh;
        ay[i] = (r[2 * i + 1] - y) * invh;
    }
    const S area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
    if (area2 == 0.0) return;
    S c[10];
    taylor_shift<ORDER, S>(r + 6, ax[0], ay[0], c);
    S bx[3], by[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j1 = i == 2 ? 0 : i + 1, j2 = i == 0 ? 2 : i - 1;
        bx[i] = rot == 0 ? ax[i] : (rot == 1 ? ax[j1] : ax[j2]);
        by[i] = rot == 0 ? ay[i] : (rot == 1 ? ay[j1] : ay[j2]);
    }
    pair_core<DEG, ORDER, S, M, EDGE_UNROLL>(K, math, tau, bx, by, area2, c, invh, oI, oX, oY);
}

// The pair for NF fields given as polynomials about the particle:
// A_f(x + h xi) = sum c[10 f + k] xi^k (record order), vertices (ax, ay) in
// units of h relative to the particle, area2 their doubled signed area
// (non-zero).  The fields share every geometric term; only the contraction
// with each field's harmonics is repeated.  EDGE_UNROLL = 1 keeps the edge
// loop rolled (one edge's state live at a time), 3 unrolls it.
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL, int NF, typename KA>
__host__ __device__ inline void pair_core_n(const KA &K, const M &math, double tau, const S *ax, const S *ay,
                                            const S &area2, const S *c, double invh, S *oI, S *oX, S *oY) {
    Harm<S> hg[NF][ORDER + 1];
#pragma unroll
    for (int f = 0; f < NF; ++f) global_harmonics<ORDER, S>(c + 10 * f, hg[f]);
    S I[NF], GX[NF], GY[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) I[f] = GX[f] = GY[f] = 0.0;
    // the vertex registers rotate, so that the loop body is the same for every edge
    S x0 = ax[0], y0 = ay[0], x1 = ax[1], y1 = ay[1], x2 = ax[2], y2 = ay[2];
    S q0 = x0 * x0 + y0 * y0, q1 = x1 * x1 + y1 * y1, q2 = x2 * x2 + y2 * y2;   // squared radii
    int skipped = 0;
#pragma unroll EDGE_UNROLL
    for (int e = 0; e < 3; ++e) {
        const S xa = x0, ya0 = y0, xb = x1, yb0 = y1, ra2 = q0, rb2 = q1;
        {
            const S rx = x0, ry = y0, rq = q0;
            x0 = x1; y0 = y1; x1 = x2; y1 = y2; x2 = rx; y2 = ry;
            q0 = q1; q1 = q2; q2 = rq;
        }
        S p, nx, ny, ya, yb;
        if (!edge_frame(math, xa, ya0, xb, yb0, p, nx, ny, ya, yb)) {
            skipped |= 1 << e;
            continue;
        }
        // harmonics in the edge frame: theta = psi + phi, (cos phi, sin phi) = n
        S cph[4], sph[4];
        edge_phases(nx, ny, cph, sph);
        Harm<S> hl[NF][ORDER + 1];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m <= ORDER; ++m)
#pragma unroll
                for (int n = 0; n < 5; ++n) {
                    if (n > 3) { hl[f][m].c[n] = hl[f][m].s[n] = 0.0; continue; }
                    const S hc = hg[f][m].c[n], hs = hg[f][m].s[n];
                    hl[f][m].c[n] = hc * cph[n] + hs * sph[n];
                    hl[f][m].s[n] = hs * cph[n] - hc * sph[n];
                }
        FieldSink<S, NF> sk;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            sk.hv[f] = hl[f];
            sk.I[f] = sk.X[f] = sk.Y[f] = 0.0;
        }
        const auto em = math.for_edge(p, tau);
        for (int pc = 0; pc < K.npieces; ++pc) edge_piece<DEG, ORDER, S>(K, em, pc, p, ya, yb, ra2, rb2, sk);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            I[f] += sk.I[f];
            GX[f] += sk.X[f] * nx - sk.Y[f] * ny;
            GY[f] += sk.X[f] * ny + sk.Y[f] * nx;
        }
    }
    // an edge skipped (particle on its line, or zero length) leaves the ray
    // terms of its neighbours at its two vertices without partners
    if (skipped) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            // vertex v starts edge v and ends edge v-1
            const bool out = skipped & (1 << v), in = skipped & (1 << (v == 0 ? 2 : v - 1));
            if (out != in)
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    vertex_ray_terms<ORDER, S>(K, math, hg[f], ax[v], ay[v], out ? 1.0 : -1.0, I[f], GX[f], GY[f]);
        }
    }
    const double sg = area2 > 0.0 ? K.cd : -K.cd;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        oI[f] = sg * I[f];
        oX[f] = -sg * invh * GX[f];
        oY[f] = -sg * invh * GY[f];
    }
}

// The pair for one field.
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL, typename KA>
__host__ __device__ inline void pair_core(const KA &K, const M &math, double tau, const S *ax, const S *ay,
                                          const S &area2, const S *c, double invh, S &oI, S &oX, S &oY) {
    pair_core_n<DEG, ORDER, S, M, EDGE_UNROLL, 1>(K, math, tau, ax, ay, area2, c, invh, &oI, &oX, &oY);
}

// ----------------------------------------------------------------------------
// adjoint of the pair with respect to the field
// ----------------------------------------------------------------------------

// Transpose of taylor_shift: weights g on the coefficients about the particle
// -> weights ge on the record's coefficients about vertex 0.
template <int ORDER, typename S>
__host__ __device__ inline void taylor_shift_T(const S *g, S sx, S sy, S *ge) {
    const S mx[4] = {1.0, -sx, sx * sx, -sx * sx * sx};
    const S my[4] = {1.0, -sy, sy * sy, -sy * sy * sy};
    constexpr double B[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
#pragma unroll
    for (int k = 0; k < 10; ++k) ge[k] = 0.0;
#pragma unroll
    for (int mi = 0; mi <= ORDER; ++mi)
#pragma unroll
        for (int j = 0; j <= mi; ++j) {
            const int i = mi - j;
            S acc = 0.0;
#pragma unroll
            for (int a = 0; a <= i; ++a)
#pragma unroll
                for (int b = 0; b <= j; ++b) {
                    const double w = B[i][a] * B[j][b];
                    const S f = w == 1.0 ? g[pidx(a, b)] : S(g[pidx(a, b)] * lit(w));
                    acc += f * mx[i - a] * my[j - b];
                }
            ge[pidx(i, j)] = acc;
        }
}

// Transpose of vertex_ray_terms with respect to the global harmonics:
// adds cI dI/dhg - (1/h) (cX dGX/dhg + cY dGY/dhg) to the weights dg.
template <int ORDER>
__device__ inline void vertex_ray_dual(const KArgs &K, double vx, double vy, double s, double invh, double cI,
                                       double cX, double cY, Harm<double> *dg) {
    using S = double;
    const S r2 = vx * vx + vy * vy;
    if (!(r2 > 0.0)) return;
    const S ir = rsqrt_nr(r2);
    const S c1 = vx * ir, s1 = vy * ir;
    Harm<S> f;                                      // c: sin(n theta)/n, s: -cos(n theta)/n
    {
        S cn1 = 1.0, sn1 = 0.0, cn = c1, sn = s1;
        f.c[0] = f.s[0] = 0.0;
#pragma unroll
        for (int n = 1; n <= ORDER + 1; ++n) {
            const double inv = lit(1.0 / n);
            f.c[n] = sn * inv;
            f.s[n] = -cn * inv;
            const S cn2 = 2.0 * c1 * cn - cn1, sn2 = 2.0 * c1 * sn - sn1;
            cn1 = cn; sn1 = sn; cn = cn2; sn = sn2;
        }
#pragma unroll
        for (int n = ORDER + 2; n < 5; ++n) f.c[n] = f.s[n] = 0.0;
    }
    for (int pc = 0; pc < K.npieces; ++pc) {
        if (!(r2 > K.R[pc] * K.R[pc])) continue;
#pragma unroll
        for (int m = 0; m <= ORDER; ++m) {
            const double wv = s * cI * K.sv[pc][m];
            const double wx = -s * invh * cX * K.sw[pc][m], wy = -s * invh * cY * K.sw[pc][m];
            Harm<S> gx, gy, d;
#pragma unroll
            for (int n = 0; n < 5; ++n) {
                gx.c[n] = wx * f.c[n];
                gx.s[n] = wx * f.s[n];
                gy.c[n] = wy * f.c[n];
                gy.s[n] = wy * f.s[n];
                d.c[n] = wv * f.c[n];
                d.s[n] = wv * f.s[n];
            }
            // the value part uses only the slots n >= 1 of A_m itself
            d.c[0] = d.s[0] = 0.0;
            // the gradient part uses the slots n >= 1 of A_m cos, A_m sin
            gx.c[0] = gx.s[0] = gy.c[0] = gy.s[0] = 0.0;
            mul_cs_T(m, gx, gy, d);
#pragma unroll
            for (int n = m & 1; n <= m; n += 2) {
                dg[m].c[n] += d.c[n];
                dg[m].s[n] += d.s[n];
            }
        }
    }
}

// Moments mom[k] = int_T xi^k Phi dxi (record order of the monomials about the
// particle, xi in units of h, with the c_d and 1/h factors of pair_core) of the
// cotangent-weighted kernel Phi = cI W + cX dW/dx_p + cY dW/dy_p; that is,
// mom[k] = cI oI + cX oX + cY oY of pair_core for the unit monomial field k.
// pair_core is linear in the field's harmonics, so one pass collects, per
// edge, the closed-form integrals of every harmonic slot (BasisSink), weights
// them with the cotangents, and carries the weights back through the product
// with (cos, sin), the edge rotation and the monomial-to-harmonic map.
//
// The same radial terms give the boundary line integrals of the transport
// term (LineSums): gv[2k], gv[2k+1] receive the line part of the gradient with
// respect to vertex k (world units), for the field c about the particle
// (units of h, record order).
//
// M is the precision policy of the square roots, reciprocals and angles
// (ExactMath, or MixedMath with its FP64 islands within tau of an edge line).
template <int DEG, int ORDER, int EDGE_UNROLL = 3, typename M = ExactMath, typename KA = KArgs>
__device__ inline void pair_dual(const KA &K, const double *ax, const double *ay, double area2, double invh,
                                 double cI, double cX, double cY, const double *c, double *mom, double *gv,
                                 const M &math = M(), double tau = 0.0) {
    using S = double;
#pragma unroll
    for (int k = 0; k < 6; ++k) gv[k] = 0.0;
    // adds the line integrals of edge e (vertex e to e+1) times the outward normal
    auto add_line = [&](int e, S Ja, S Jb, S ox, S oy) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const S w = k == e ? Ja : (k == (e == 2 ? 0 : e + 1) ? Jb : S(0.0));
            gv[2 * k] = fma(w, ox, gv[2 * k]);
            gv[2 * k + 1] = fma(w, oy, gv[2 * k + 1]);
        }
    };
    const double so = area2 > 0.0 ? 1.0 : -1.0;
    Harm<S> dg[ORDER + 1];          // weights of the global-frame harmonics
#pragma unroll
    for (int m = 0; m <= ORDER; ++m)
#pragma unroll
        for (int n = 0; n < 5; ++n) dg[m].c[n] = dg[m].s[n] = 0.0;
    S x0 = ax[0], y0 = ay[0], x1 = ax[1], y1 = ay[1], x2 = ax[2], y2 = ay[2];
    S q0 = x0 * x0 + y0 * y0, q1 = x1 * x1 + y1 * y1, q2 = x2 * x2 + y2 * y2;   // squared radii
    int skipped = 0;
#pragma unroll EDGE_UNROLL
    for (int e = 0; e < 3; ++e) {
        const S xa = x0, ya0 = y0, xb = x1, yb0 = y1, ra2 = q0, rb2 = q1;
        {
            const S rx = x0, ry = y0, rq = q0;
            x0 = x1; y0 = y1; x1 = x2; y1 = y2; x2 = rx; y2 = ry;
            q0 = q1; q1 = q2; q2 = rq;
        }
        S p, nx, ny, ya, yb;
        if (!edge_frame(math, xa, ya0, xb, yb0, p, nx, ny, ya, yb)) {
            skipped |= 1 << e;
            const S Lx = xb - xa, Ly = yb0 - ya0;
            const S len2 = Lx * Lx + Ly * Ly;
            if (len2 != 0.0) {
                // the edge lies on a line through the particle: y along the
                // edge (tau = t, normal (ty, -tx))
                S len, il;
                math.edge_norm(len2, len, il);
                const S tx = Lx * il, ty = Ly * il;
                const S la = xa * tx + ya0 * ty, lb = la + len;
                LineSink<DEG, ORDER, S> ls;
                ls.ln.clear();
#pragma unroll
                for (int pc = 0; pc < 2; ++pc)
                    if (pc < K.npieces) edge_piece<DEG, ORDER, S>(K, math.for_edge(0.0, tau), pc, S(0.0), la, lb, ra2,
                                                                  rb2, ls);
                S Ja, Jb;
                ls.ln.finish(S(0.0), la, lb, ty, -tx, c, cI, cX, cY, invh, K.cd, Ja, Jb);
                add_line(e, Ja, Jb, so * ty, -so * tx);
            }
            continue;
        }
        BasisLineSink<DEG, ORDER, S> sk;
        sk.ln.clear();
#pragma unroll
        for (int m = 0; m <= ORDER; ++m)
#pragma unroll
            for (int n = 0; n < 5; ++n) sk.vb[m].c[n] = sk.vb[m].s[n] = sk.gb[m].c[n] = sk.gb[m].s[n] = 0.0;
        // pieces unrolled (at most two): a constant piece index keeps every
        // coefficient a scalar load from the argument block
        const auto em = math.for_edge(p, tau);
#pragma unroll
        for (int pc = 0; pc < 2; ++pc)
            if (pc < K.npieces) edge_piece<DEG, ORDER, S>(K, em, pc, p, ya, yb, ra2, rb2, sk);
        // the edge's share of cI I + cX GX + cY GY in the edge frame:
        // cI eI - (1/h) (gn eX + gt eY), (gn, gt) = cotangent in (n, t)
        const S wX = -invh * (cX * nx + cY * ny), wY = -invh * (cY * nx - cX * ny);
        S cph[4], sph[4];
        edge_phases(nx, ny, cph, sph);
#pragma unroll
        for (int m = 0; m <= ORDER; ++m) {
            Harm<S> gx, gy, d;
#pragma unroll
            for (int n = 0; n < 5; ++n) {
                gx.c[n] = wX * sk.gb[m].c[n];
                gx.s[n] = wX * sk.gb[m].s[n];
                gy.c[n] = wY * sk.gb[m].c[n];
                gy.s[n] = wY * sk.gb[m].s[n];
                d.c[n] = cI * sk.vb[m].c[n];
                d.s[n] = cI * sk.vb[m].s[n];
            }
            mul_cs_T(m, gx, gy, d);
            // transpose of the rotation into the edge frame
#pragma unroll
            for (int n = m & 1; n <= m; n += 2) {
                dg[m].c[n] += d.c[n] * cph[n] - d.s[n] * sph[n];
                dg[m].s[n] += d.c[n] * sph[n] + d.s[n] * cph[n];
            }
        }
        // line integrals; the outward normal (ty, -tx) so, with (ty, -tx) =
        // +-(nx, ny) as yb > ya or not
        {
            S Ja, Jb;
            sk.ln.finish(p, ya, yb, nx, ny, c, cI, cX, cY, invh, K.cd, Ja, Jb);
            const S o = (yb > ya) == (area2 > 0.0) ? 1.0 : -1.0;
            add_line(e, Ja, Jb, o * nx, o * ny);
        }
    }
    // ray terms at the vertices of skipped edges (see pair_core), in the
    // triangle's frame: weights of the global harmonics directly
    if (skipped) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const bool out = skipped & (1 << v), in = skipped & (1 << (v == 0 ? 2 : v - 1));
            if (out != in) vertex_ray_dual<ORDER>(K, ax[v], ay[v], out ? 1.0 : -1.0, invh, cI, cX, cY, dg);
        }
    }
    // transpose of global_harmonics, times the orientation sign and c_d
    const double sg = area2 > 0.0 ? K.cd : -K.cd;
    mom[0] = sg * dg[0].c[0];
    if (ORDER >= 1) {
        mom[pidx(1, 0)] = sg * dg[1].c[1];
        mom[pidx(0, 1)] = sg * dg[1].s[1];
    }
    if (ORDER >= 2) {
        mom[pidx(2, 0)] = 0.5 * sg * (dg[2].c[0] + dg[2].c[2]);
        mom[pidx(0, 2)] = 0.5 * sg * (dg[2].c[0] - dg[2].c[2]);
        mom[pidx(1, 1)] = 0.5 * sg * dg[2].s[2];
    }
    if (ORDER >= 3) {
        mom[pidx(3, 0)] = lit(0.25) * sg * fma(lit(3.0), dg[3].c[1], dg[3].c[3]);
        mom[pidx(1, 2)] = lit(0.25) * sg * (dg[3].c[1] - dg[3].c[3]);
        mom[pidx(2, 1)] = lit(0.25) * sg * (dg[3].s[1] + dg[3].s[3]);
        mom[pidx(0, 3)] = lit(0.25) * sg * fma(lit(3.0), dg[3].s[1], -dg[3].s[3]);
    }
}

}  // namespace sphbi
