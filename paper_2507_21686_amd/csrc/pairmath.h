// Closed-form pair mathematics shared by the forward and adjoint kernels.
// Templated on the scalar type S: double for the forward path, a
// forward-mode dual number for the adjoint (derivatives with respect to the
// triangle vertices propagate through every step, including the clipping).
// See forward.hip for the derivation.
#pragma once

#include <math.h>

#include "internal.h"
#include "precision.h"

namespace sphbi {

__host__ __device__ constexpr int pidx(int i, int j) { return (i + j) * (i + j + 1) / 2 + j; }

// An FP64 constant as an instruction operand: the values the hardware encodes
// inline (0, +-1/2, +-1, +-2, +-4) stay literal, every other one is handed
// over through a scalar register at its point of use (see sconst()).
__device__ inline double lit(double c) {
    const double a = fabs(c);
    return (a == 0.0 || a == 0.5 || a == 1.0 || a == 2.0 || a == 4.0) ? c : sconst(c);
}

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

// One record: vertices v[6] (world units) and nodal values A[n_nodes] ->
// rec[16] = v, then e_ij of A(v0 + h eta) = sum e_ij eta_x^i eta_y^j.
template <int ORDER, typename S>
__host__ __device__ inline void prepare_record(const S *v, const S *A, double invh, S *r) {
    S e[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) e[k] = 0.0;
    if (ORDER == 0) {
        e[0] = A[0];
    } else {
        const S q1x = (v[2] - v[0]) * invh, q1y = (v[3] - v[1]) * invh;
        const S q2x = (v[4] - v[0]) * invh, q2y = (v[5] - v[1]) * invh;
        const S det = q1x * q2y - q1y * q2x;
        if (det != 0.0) {
            const S id = 1.0 / det;
            // barycentric coordinates as affine forms in eta (origin at v0)
            const S l1x = q2y * id, l1y = -q2x * id;
            const S l2x = -q1y * id, l2y = q1x * id;
            const S la[3] = {1.0, 0.0, 0.0};
            const S lx[3] = {-(l1x + l2x), l1x, l2x};
            const S ly[3] = {-(l1y + l2y), l1y, l2y};
            if (ORDER == 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    e[0] += A[i] * la[i];
                    e[1] += A[i] * lx[i];
                    e[2] += A[i] * ly[i];
                }
            } else {
                S one[10], t1[10], t2[10], t3[10];
#pragma unroll
                for (int k = 0; k < 10; ++k) one[k] = k == 0 ? 1.0 : 0.0;
                // vertices: lambda (3 lambda - 1)(3 lambda - 2) / 2
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    mul_affine(one, la[i], lx[i], ly[i], t1);
                    mul_affine(t1, 3.0 * la[i] - 1.0, 3.0 * lx[i], 3.0 * ly[i], t2);
                    mul_affine(t2, 3.0 * la[i] - 2.0, 3.0 * lx[i], 3.0 * ly[i], t3);
#pragma unroll
                    for (int k = 0; k < 10; ++k) e[k] += 0.5 * A[i] * t3[k];
                }
                // edge nodes: 9/2 lambda_a lambda_b (3 lambda_a - 1) at 1/3 from a,
                //             9/2 lambda_a lambda_b (3 lambda_b - 1) at 2/3 from a
#pragma unroll
                for (int ed = 0; ed < 3; ++ed) {
                    const int a = ed, b = (ed + 1) % 3;
                    mul_affine(one, la[a], lx[a], ly[a], t1);
                    mul_affine(t1, la[b], lx[b], ly[b], t2);
                    mul_affine(t2, 3.0 * la[a] - 1.0, 3.0 * lx[a], 3.0 * ly[a], t3);
#pragma unroll
                    for (int k = 0; k < 10; ++k) e[k] += 4.5 * A[3 + 2 * ed] * t3[k];
                    mul_affine(t2, 3.0 * la[b] - 1.0, 3.0 * lx[b], 3.0 * ly[b], t3);
#pragma unroll
                    for (int k = 0; k < 10; ++k) e[k] += 4.5 * A[4 + 2 * ed] * t3[k];
                }
                // centroid: 27 lambda_0 lambda_1 lambda_2
                mul_affine(one, la[0], lx[0], ly[0], t1);
                mul_affine(t1, la[1], lx[1], ly[1], t2);
                mul_affine(t2, la[2], lx[2], ly[2], t3);
#pragma unroll
                for (int k = 0; k < 10; ++k) e[k] += 27.0 * A[9] * t3[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) r[k] = v[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) r[6 + k] = e[k];
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

// One edge of the signed fan, one kernel piece of radius R.  Adds the
// edge-frame value and gradient integrals (without c_d and without the
// -1/h of the gradient).
template <int DEG, int ORDER, typename S, typename M>
__host__ __device__ inline void edge_piece(const KArgs &K, const M &math, int pc, S p, S ya, S yb,
                                           const Harm<S> *hv, S &oI, S &oX, S &oY) {
    constexpr int HMAX = DEG + ORDER + 1;
    constexpr int PMAX = DEG + ORDER;
    const double R = K.R[pc];
    const S yc = p < R ? S(math.sqrt_((R - p) * (R + p))) : S(0.0);
    const S aya = fabs(ya), ayb = fabs(yb);
    const bool clipA = aya > yc, clipB = ayb > yc;

    // ---- sector parts of clipped endpoints (cone formulas, Sec. 5.2)
    S angc[5], angs[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) angc[n] = angs[n] = 0.0;
    const S cpc = p < R ? S(p * K.iR[pc]) : S(1.0), spc = p < R ? S(yc * K.iR[pc]) : S(0.0);   // (cos, sin) psi_c
#pragma unroll
    for (int end = 0; end < 2; ++end) {
        const bool clip = end ? clipB : clipA;
        if (!clip) continue;
        const S y = end ? yb : ya, ay = end ? ayb : aya;
        const double sg = end ? 1.0 : -1.0;          // Q(y_b) - Q(y_a)
        const double sy = y > 0.0 ? sg : -sg;          // odd cosine part
        S ir, ang;
        math.sector_seed(p, ay, yc, ir, ang);
        const S cu = p * ir, su = ay * ir;
        angc[0] += sy * ang;
        S cn1 = 1.0, sn1 = 0.0, cn = cu, sn = su;      // cos/sin of n u
        S dn1 = 1.0, tn1 = 0.0, dn = cpc, tn = spc;    // cos/sin of n psi_c
#pragma unroll
        for (int n = 1; n <= ORDER + 1; ++n) {
            const double inv = lit(1.0 / n);
            const double sinv = sy * inv, ginv = sg * inv;
            angc[n] += (sn - tn) * sinv;
            angs[n] += (dn - cn) * ginv;
            const S cn2 = 2.0 * cu * cn - cn1, sn2 = 2.0 * cu * sn - sn1;
            const S dn2 = 2.0 * cpc * dn - dn1, tn2 = 2.0 * cpc * tn - tn1;
            cn1 = cn; sn1 = sn; cn = cn2; sn = sn2;
            dn1 = dn; tn1 = tn; dn = dn2; tn = tn2;
        }
    }
    // contract the sector parts now, so that the angular terms are dead
    // before the radial terms are formed
    if (clipA || clipB) {
#pragma unroll
        for (int m = 0; m <= ORDER; ++m) {
            Harm<S> hx, hy;
            mul_cs(m, hv[m], hx, hy);
            const double sv = K.sv[pc][m], sw = K.sw[pc][m];
#pragma unroll
            for (int n = m & 1; n <= m; n += 2) oI += sv * (hv[m].c[n] * angc[n] + hv[m].s[n] * angs[n]);
#pragma unroll
            for (int n = (m + 1) & 1; n <= m + 1; n += 2) {
                oX += sw * (hx.c[n] * angc[n] + hx.s[n] * angs[n]);
                oY += sw * (hy.c[n] * angc[n] + hy.s[n] * angs[n]);
            }
        }
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
        H[0] = h0;
        H[1] = yB - yA;
        S gA = 1.0, gB = 1.0;          // rho^{c-1}
#pragma unroll
        for (int c = 2; c <= HMAX; ++c) {
            gA *= rA;
            gB *= rB;
            H[c] = (gB * yB - gA * yA + lit(c - 1.0) * p2 * H[c - 2]) * lit(1.0 / c);
        }
        S qA = rA, qB = rB;            // rho^{e+1}
#pragma unroll
        for (int e = 0; e <= PMAX; ++e) {
            P[e] = (qB - qA) * lit(1.0 / (e + 1));
            qA *= rA;
            qB *= rB;
        }
    }
    S pj[ORDER + 3];
    pj[0] = p;                             // p^{j+1}
#pragma unroll
    for (int j = 1; j < ORDER + 3; ++j) pj[j] = pj[j - 1] * p;

#pragma unroll
    for (int m = 0; m <= ORDER; ++m) {
        Harm<S> hx, hy;
        mul_cs(m, hv[m], hx, hy);
        // kernel-contracted radial sums
        S Ac[ORDER + 1], As[ORDER + 1], Bc[ORDER + 2], Bs[ORDER + 1];
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 0; k <= DEG; ++k) s = fma(K.bq[pc][m][k], H[k + 1 + m - j], s);
            Ac[j] = s;
        }
#pragma unroll
        for (int j = 0; j < m; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 0; k <= DEG; ++k) s = fma(K.bq[pc][m][k], P[k + m - j], s);
            As[j] = s;
        }
#pragma unroll
        for (int j = 0; j <= m + 1; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 1; k <= DEG; ++k) s = fma(K.kbq[pc][m][k], H[k + m - j], s);
            Bc[j] = s;
        }
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            S s = 0.0;
#pragma unroll
            for (int k = 1; k <= DEG; ++k) s = fma(K.kbq[pc][m][k], P[k + m - 1 - j], s);
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
            oI += hv[m].c[n] * vc + hv[m].s[n] * vs;
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
            oX += hx.c[n] * wc + hx.s[n] * ws;
            oY += hy.c[n] * wc + hy.s[n] * ws;
        }
    }
}

// tau: edges whose line passes within tau (units of h) of the particle are
// evaluated with the exact policy (only meaningful for MixedMath).
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL = 3>
__host__ __device__ inline void pair_core(const KArgs &K, const M &math, double tau, const S *ax, const S *ay,
                                          const S &area2, const S *c, double invh, S &oI, S &oX, S &oY);

// One pair: particle (x, y), record r (vertices and field about vertex 0).
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL = 3>
__host__ __device__ inline void pair_fwd(const KArgs &K, const M &math, double tau, S x, S y, double invh,
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

// The pair for a field given as a polynomial about the particle:
// A(x + h xi) = sum c_ij xi_x^i xi_y^j, vertices (ax, ay) in units of h
// relative to the particle, area2 their doubled signed area (non-zero).
// EDGE_UNROLL = 1 keeps the edge loop rolled (one edge's state live at a
// time), 3 unrolls it.
template <int DEG, int ORDER, typename S, typename M, int EDGE_UNROLL>
__host__ __device__ inline void pair_core(const KArgs &K, const M &math, double tau, const S *ax, const S *ay,
                                          const S &area2, const S *c, double invh, S &oI, S &oX, S &oY) {
    Harm<S> hg[ORDER + 1];
    global_harmonics<ORDER, S>(c, hg);
    S I = 0.0, GX = 0.0, GY = 0.0;
    // the vertex registers rotate, so that the loop body is the same for every edge
    S x0 = ax[0], y0 = ay[0], x1 = ax[1], y1 = ay[1], x2 = ax[2], y2 = ay[2];
#pragma unroll EDGE_UNROLL
    for (int e = 0; e < 3; ++e) {
        const S axe = x0, aye = y0;
        const S Lx = x1 - axe, Ly = y1 - aye;
        {
            const S rx = x0, ry = y0;
            x0 = x1; y0 = y1; x1 = x2; y1 = y2; x2 = rx; y2 = ry;
        }
        const S len2 = Lx * Lx + Ly * Ly;
        if (len2 == 0.0) continue;
        S len, il;
        math.edge_norm(len2, len, il);
        const S tx = Lx * il, ty = Ly * il;
        const S sd = axe * ty - aye * tx;        // signed distance of the edge line
        const S p = fabs(sd);
        if (p == 0.0) continue;                       // fan triangle of zero area
        const S nx = sd > 0.0 ? ty : S(-ty), ny = sd > 0.0 ? S(-tx) : tx;
        const S ya = -axe * ny + aye * nx;       // along-edge coordinates from the foot
        const S yb = sd > 0.0 ? S(ya + len) : S(ya - len);
        // harmonics in the edge frame: theta = psi + phi, (cos phi, sin phi) = n
        Harm<S> hl[ORDER + 1];
        S cph[4], sph[4];
        cph[0] = 1.0; sph[0] = 0.0;
        cph[1] = nx; sph[1] = ny;
#pragma unroll
        for (int n = 2; n <= 3; ++n) {
            cph[n] = 2.0 * nx * cph[n - 1] - cph[n - 2];
            sph[n] = 2.0 * nx * sph[n - 1] - sph[n - 2];
        }
#pragma unroll
        for (int m = 0; m <= ORDER; ++m)
#pragma unroll
            for (int n = 0; n < 5; ++n) {
                if (n > 3) { hl[m].c[n] = hl[m].s[n] = 0.0; continue; }
                const S hc = hg[m].c[n], hs = hg[m].s[n];
                hl[m].c[n] = hc * cph[n] + hs * sph[n];
                hl[m].s[n] = hs * cph[n] - hc * sph[n];
            }
        S eI = 0.0, eX = 0.0, eY = 0.0;
        const auto em = math.for_edge(p, tau);
        for (int pc = 0; pc < K.npieces; ++pc) edge_piece<DEG, ORDER, S>(K, em, pc, p, ya, yb, hl, eI, eX, eY);
        I += eI;
        GX += eX * nx - eY * ny;
        GY += eX * ny + eY * nx;
    }
    const double sg = area2 > 0.0 ? K.cd : -K.cd;
    oI = sg * I;
    oX = -sg * invh * GX;
    oY = -sg * invh * GY;
}

}  // namespace sphbi
