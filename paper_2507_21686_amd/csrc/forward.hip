// Forward pair kernel: closed-form int_T A W and int_T A grad W for every
// (particle, triangle) pair, summed per particle.
//
// Decomposition (Sec. 4, eq. intermediateWedge): with the particle at the
// origin of the support-normalised frame (Sec. 2, transform C), a triangle
// with vertices a0, a1, a2 is the signed sum of the three particle-anchored
// triangles (0, a_e, a_{e+1}), each weighted by the sign of its area.  In
// the frame of an edge (x' along the unit normal n towards the edge line at
// distance p, y' along the edge) that triangle is
//     { psi in [psi_a, psi_b], 0 <= r <= min(R, p / cos psi) },
// i.e. the difference of two right-angled stubs anchored at the foot of the
// perpendicular, Q(y_b) - Q(y_a), where each stub is a sector beyond the
// circle crossing and a triangle inside it (Sec. 4.3).  Rotating the field
// into the edge frame is the improper-rotation rule (eq. improper) applied to
// every harmonic at once.
//
// Closed forms (Sec. 5).  For the triangle part of a stub the substitution
// r = p / cos psi turns every moment into radial integrals with Chebyshev
// angular factors (Sec. 5.1):
//     int_0^u cos(n psi) (p/cos psi)^{K+1} dpsi/(K+1)
//         = p/(K+1) sum_j T_n[j] p^j  H_{K-j},
//     int_0^u sin(n psi) (p/cos psi)^{K+1} dpsi/(K+1)
//         = p/(K+1) sum_j U_{n-1}[j] p^j  P_{K-1-j},
// with the hypergeometric radial term H_c = int_p^rho r^c (r^2-p^2)^{-1/2} dr
// (a 2F1 of argument (p/r)^2) evaluated by the contiguous relation
// c H_c = rho^{c-1} y + (c-1) p^2 H_{c-2} from H_0 = asinh(y/p), H_1 = y --
// every term is positive, so the recurrence is stable -- and the powers
// P_e = int_p^rho r^e dr.  The sector parts are the cone formulas of
// Sec. 5.2.  The kernel (Sec. 2, k = sum b_k q^k) and the field harmonics
// (Sec. 3, Table 1 with the gradient of eq. basicdiff) are contracted with
// these radial terms per edge.
//
// Work layout: a wavefront owns 64 consecutive particles; its lanes sweep the
// particles' CSR pair range 64 pairs at a time (one pair per lane), and a
// segmented wave scan (pairs of a particle are contiguous) sums each
// particle's pairs in a fixed order, so the result is deterministic without
// atomics.

#include <math.h>

#include "internal.h"

namespace sphbi {
namespace {

__host__ __device__ constexpr int pidx(int i, int j) { return (i + j) * (i + j + 1) / 2 + j; }

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
__host__ __device__ inline void mul_affine(const double *in, double a, double bx, double by, double *out) {
#pragma unroll
    for (int m = 0; m <= 3; ++m)
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            const int i = m - j;
            double v = a * in[pidx(i, j)];
            if (i > 0) v += bx * in[pidx(i - 1, j)];
            if (j > 0) v += by * in[pidx(i, j - 1)];
            out[pidx(i, j)] = v;
        }
}

// One record: vertices v[6] (world units) and nodal values A[n_nodes] ->
// rec[16] = v, then e_ij of A(v0 + h eta) = sum e_ij eta_x^i eta_y^j.
template <int ORDER>
__host__ __device__ inline void prepare_record(const double *v, const double *A, double invh, double *r) {
    double e[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) e[k] = 0.0;
    if (ORDER == 0) {
        e[0] = A[0];
    } else {
        const double q1x = (v[2] - v[0]) * invh, q1y = (v[3] - v[1]) * invh;
        const double q2x = (v[4] - v[0]) * invh, q2y = (v[5] - v[1]) * invh;
        const double det = q1x * q2y - q1y * q2x;
        if (det != 0.0) {
            const double id = 1.0 / det;
            // barycentric coordinates as affine forms in eta (origin at v0)
            const double l1x = q2y * id, l1y = -q2x * id;
            const double l2x = -q1y * id, l2y = q1x * id;
            const double la[3] = {1.0, 0.0, 0.0};
            const double lx[3] = {-(l1x + l2x), l1x, l2x};
            const double ly[3] = {-(l1y + l2y), l1y, l2y};
            if (ORDER == 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    e[0] += A[i] * la[i];
                    e[1] += A[i] * lx[i];
                    e[2] += A[i] * ly[i];
                }
            } else {
                double one[10], t1[10], t2[10], t3[10];
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

template <int ORDER>
__global__ __launch_bounds__(256) void prepare_kernel(int64_t T, const double *__restrict__ tri,
                                                      const double *__restrict__ nodal, double invh,
                                                      double *__restrict__ rec) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
    double v[6], A[10];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
#pragma unroll
    for (int k = 0; k < 10; ++k) A[k] = k < NN ? nodal[k * T + t] : 0.0;
    double r[kRecDoubles];
    prepare_record<ORDER>(v, A, invh, r);
    double *o = rec + t * kRecDoubles;
#pragma unroll
    for (int k = 0; k < kRecDoubles; ++k) o[k] = r[k];
}

// ----------------------------------------------------------------------------
// per-pair closed form
// ----------------------------------------------------------------------------

// Harmonics of a degree-m homogeneous part: A_m(psi) = sum_n hc[n] cos(n psi) + hs[n] sin(n psi)
struct Harm {
    double c[5], s[5];
};

// A_m(psi) * cos(psi) and A_m(psi) * sin(psi) (product-to-sum)
__host__ __device__ inline void mul_cs(int M, const Harm &v, Harm &x, Harm &y) {
#pragma unroll
    for (int n = 0; n < 5; ++n) { x.c[n] = x.s[n] = y.c[n] = y.s[n] = 0.0; }
#pragma unroll
    for (int n = M & 1; n <= M; n += 2) {
        const double c = v.c[n], s = v.s[n];
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

template <int ORDER>
__host__ __device__ inline void global_harmonics(const double *c, Harm *h) {
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
        const double c20 = c[pidx(2, 0)], c11 = c[pidx(1, 1)], c02 = c[pidx(0, 2)];
        h[2].c[0] = 0.5 * (c20 + c02);
        h[2].c[2] = 0.5 * (c20 - c02);
        h[2].s[2] = 0.5 * c11;
    }
    if (ORDER >= 3) {
        const double c30 = c[pidx(3, 0)], c21 = c[pidx(2, 1)], c12 = c[pidx(1, 2)], c03 = c[pidx(0, 3)];
        h[3].c[1] = 0.25 * (3.0 * c30 + c12);
        h[3].s[1] = 0.25 * (c21 + 3.0 * c03);
        h[3].c[3] = 0.25 * (c30 - c12);
        h[3].s[3] = 0.25 * (c21 - c03);
    }
}

// A(xi) = sum e_ij (xi - s)^(i,j): coefficients about the particle
template <int ORDER>
__host__ __device__ inline void taylor_shift(const double *__restrict__ e, double sx, double sy, double *c) {
    // powers of -s
    const double mx[4] = {1.0, -sx, sx * sx, -sx * sx * sx};
    const double my[4] = {1.0, -sy, sy * sy, -sy * sy * sy};
    constexpr double B[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
#pragma unroll
    for (int k = 0; k < 10; ++k) c[k] = 0.0;
#pragma unroll
    for (int mi = 0; mi <= ORDER; ++mi)
#pragma unroll
        for (int j = 0; j <= mi; ++j) {
            const int i = mi - j;
            const double eij = e[pidx(i, j)];
#pragma unroll
            for (int a = 0; a <= i; ++a)
#pragma unroll
                for (int b = 0; b <= j; ++b) c[pidx(a, b)] += eij * B[i][a] * B[j][b] * mx[i - a] * my[j - b];
        }
}

// One edge of the signed fan, one kernel piece of radius R.  Adds the
// edge-frame value and gradient integrals (without c_d and without the
// -1/h of the gradient).
template <int DEG, int ORDER>
__host__ __device__ inline void edge_piece(const KArgs &K, int pc, double p, double ya, double yb, const Harm *hv,
                                  double &oI, double &oX, double &oY) {
    constexpr int HMAX = DEG + ORDER + 1;
    constexpr int PMAX = DEG + ORDER;
    const double R = K.R[pc];
    const double yc = p < R ? sqrt((R - p) * (R + p)) : 0.0;
    const double aya = fabs(ya), ayb = fabs(yb);
    const bool clipA = aya > yc, clipB = ayb > yc;

    // ---- sector parts of clipped endpoints (cone formulas, Sec. 5.2)
    double angc[5], angs[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) angc[n] = angs[n] = 0.0;
    const double cpc = p < R ? p / R : 1.0, spc = p < R ? yc / R : 0.0;   // (cos, sin) psi_c
#pragma unroll
    for (int end = 0; end < 2; ++end) {
        const bool clip = end ? clipB : clipA;
        if (!clip) continue;
        const double y = end ? yb : ya, ay = end ? ayb : aya;
        const double sg = end ? 1.0 : -1.0;          // Q(y_b) - Q(y_a)
        const double sy = y > 0 ? sg : -sg;          // odd cosine part
        const double ir = 1.0 / sqrt(p * p + y * y);
        const double cu = p * ir, su = ay * ir;
        angc[0] += sy * atan2(p * (ay - yc), p * p + ay * yc);
        double cn1 = 1.0, sn1 = 0.0, cn = cu, sn = su;      // cos/sin of n u
        double dn1 = 1.0, tn1 = 0.0, dn = cpc, tn = spc;    // cos/sin of n psi_c
#pragma unroll
        for (int n = 1; n <= ORDER + 1; ++n) {
            const double inv = 1.0 / n;
            angc[n] += sy * (sn - tn) * inv;
            angs[n] += sg * (dn - cn) * inv;
            const double cn2 = 2.0 * cu * cn - cn1, sn2 = 2.0 * cu * sn - sn1;
            const double dn2 = 2.0 * cpc * dn - dn1, tn2 = 2.0 * cpc * tn - tn1;
            cn1 = cn; sn1 = sn; cn = cn2; sn = sn2;
            dn1 = dn; tn1 = tn; dn = dn2; tn = tn2;
        }
    }

    // ---- triangle parts: radial 2F1 terms H_c and powers P_e
    double H[HMAX + 1], P[PMAX + 1];
    const bool tri = p < R && (aya > 0.0 || ayb > 0.0);
    if (tri) {
        const double yA = clipA ? copysign(yc, ya) : ya;
        const double yB = clipB ? copysign(yc, yb) : yb;
        const double rA = clipA ? R : sqrt(p * p + ya * ya);
        const double rB = clipB ? R : sqrt(p * p + yb * yb);
        const double ip = 1.0 / p;
        const double fA = (fabs(yA) + rA) * ip, fB = (fabs(yB) + rB) * ip;
        double h0;
        // H_0 = asinh(yB/p) - asinh(yA/p) with a single logarithm
        if ((yA < 0.0 && yB > 0.0) || (yA > 0.0 && yB < 0.0)) h0 = (yB > 0.0 ? 1.0 : -1.0) * log(fA * fB);
        else if (yB != 0.0) h0 = (yB > 0.0 ? 1.0 : -1.0) * log(fB / fA);
        else h0 = (yA > 0.0 ? -1.0 : 1.0) * log(fA);
        const double p2 = p * p;
        H[0] = h0;
        H[1] = yB - yA;
        double gA = 1.0, gB = 1.0;          // rho^{c-1}
#pragma unroll
        for (int c = 2; c <= HMAX; ++c) {
            gA *= rA;
            gB *= rB;
            H[c] = (gB * yB - gA * yA + (c - 1) * p2 * H[c - 2]) * (1.0 / c);
        }
        double qA = rA, qB = rB;            // rho^{e+1}
#pragma unroll
        for (int e = 0; e <= PMAX; ++e) {
            P[e] = (qB - qA) * (1.0 / (e + 1));
            qA *= rA;
            qB *= rB;
        }
    }
    double pj[ORDER + 3];
    pj[0] = p;                             // p^{j+1}
#pragma unroll
    for (int j = 1; j < ORDER + 3; ++j) pj[j] = pj[j - 1] * p;

#pragma unroll
    for (int m = 0; m <= ORDER; ++m) {
        Harm hx, hy;
        mul_cs(m, hv[m], hx, hy);
        // sector parts
        const double sv = K.sv[pc][m], sw = K.sw[pc][m];
        if (clipA || clipB) {
#pragma unroll
            for (int n = m & 1; n <= m; n += 2) oI += sv * (hv[m].c[n] * angc[n] + hv[m].s[n] * angs[n]);
#pragma unroll
            for (int n = (m + 1) & 1; n <= m + 1; n += 2) {
                oX += sw * (hx.c[n] * angc[n] + hx.s[n] * angs[n]);
                oY += sw * (hy.c[n] * angc[n] + hy.s[n] * angs[n]);
            }
        }
        if (!tri) continue;
        // kernel-contracted radial sums
        double Ac[ORDER + 1], As[ORDER + 1], Bc[ORDER + 2], Bs[ORDER + 1];
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k <= DEG; ++k) s = fma(K.bq[pc][m][k], H[k + 1 + m - j], s);
            Ac[j] = s;
        }
#pragma unroll
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k <= DEG; ++k) s = fma(K.bq[pc][m][k], P[k + m - j], s);
            As[j] = s;
        }
#pragma unroll
        for (int j = 0; j <= m + 1; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 1; k <= DEG; ++k) s = fma(K.kbq[pc][m][k], H[k + m - j], s);
            Bc[j] = s;
        }
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 1; k <= DEG; ++k) s = fma(K.kbq[pc][m][k], P[k + m - 1 - j], s);
            Bs[j] = s;
        }
        // value harmonics n = m, m-2, ...
#pragma unroll
        for (int n = m & 1; n <= m; n += 2) {
            double vc = 0.0, vs = 0.0;
#pragma unroll
            for (int j = 0; j <= n; ++j)
                if (chebT(n, j) != 0.0) vc = fma(chebT(n, j) * pj[j], Ac[j], vc);
#pragma unroll
            for (int j = 0; j < n; ++j)
                if (chebU(n - 1, j) != 0.0) vs = fma(chebU(n - 1, j) * pj[j], As[j], vs);
            oI += hv[m].c[n] * vc + hv[m].s[n] * vs;
        }
        // gradient harmonics n = m+1, m-1, ...
#pragma unroll
        for (int n = (m + 1) & 1; n <= m + 1; n += 2) {
            double wc = 0.0, ws = 0.0;
#pragma unroll
            for (int j = 0; j <= n; ++j)
                if (chebT(n, j) != 0.0) wc = fma(chebT(n, j) * pj[j], Bc[j], wc);
#pragma unroll
            for (int j = 0; j < n; ++j)
                if (chebU(n - 1, j) != 0.0) ws = fma(chebU(n - 1, j) * pj[j], Bs[j], ws);
            oX += hx.c[n] * wc + hx.s[n] * ws;
            oY += hy.c[n] * wc + hy.s[n] * ws;
        }
    }
}

template <int DEG, int ORDER>
__host__ __device__ inline void pair_fwd(const KArgs &K, double x, double y, double invh, const double *__restrict__ r,
                                double &oI, double &oX, double &oY) {
    oI = oX = oY = 0.0;
    double ax[3], ay[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ax[i] = (r[2 * i] - x) * invh;
        ay[i] = (r[2 * i + 1] - y) * invh;
    }
    const double area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
    if (area2 == 0.0) return;
    double c[10];
    taylor_shift<ORDER>(r + 6, ax[0], ay[0], c);
    Harm hg[ORDER + 1];
    global_harmonics<ORDER>(c, hg);
    double I = 0.0, GX = 0.0, GY = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int f = e == 2 ? 0 : e + 1;
        const double axe = ax[e], aye = ay[e];
        const double Lx = ax[f] - axe, Ly = ay[f] - aye;
        const double len2 = Lx * Lx + Ly * Ly;
        if (len2 == 0.0) continue;
        const double len = sqrt(len2), il = 1.0 / len;
        const double tx = Lx * il, ty = Ly * il;
        const double sd = axe * ty - aye * tx;        // signed distance of the edge line
        const double p = fabs(sd);
        if (p == 0.0) continue;                       // fan triangle of zero area
        const double nx = sd > 0.0 ? ty : -ty, ny = sd > 0.0 ? -tx : tx;
        const double ya = -axe * ny + aye * nx;       // along-edge coordinates from the foot
        const double yb = sd > 0.0 ? ya + len : ya - len;
        // harmonics in the edge frame: theta = psi + phi, (cos phi, sin phi) = n
        Harm hl[ORDER + 1];
        double cph[4], sph[4];
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
                const double hc = hg[m].c[n], hs = hg[m].s[n];
                hl[m].c[n] = hc * cph[n] + hs * sph[n];
                hl[m].s[n] = hs * cph[n] - hc * sph[n];
            }
        double eI = 0.0, eX = 0.0, eY = 0.0;
        for (int pc = 0; pc < K.npieces; ++pc) edge_piece<DEG, ORDER>(K, pc, p, ya, yb, hl, eI, eX, eY);
        I += eI;
        GX += eX * nx - eY * ny;
        GY += eX * ny + eY * nx;
    }
    const double sg = area2 > 0.0 ? K.cd : -K.cd;
    oI = sg * I;
    oX = -sg * invh * GX;
    oY = -sg * invh * GY;
}

template <int DEG, int ORDER>
__global__ __launch_bounds__(256) void forward_kernel(const KArgs K, double invh, int64_t N,
                                                      const double *__restrict__ px,
                                                      const double *__restrict__ py,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ tri_idx,
                                                      const double *__restrict__ rec, double *__restrict__ I,
                                                      double *__restrict__ Gx, double *__restrict__ Gy,
                                                      double *__restrict__ per_pair, int64_t P, int64_t T) {
    const int lane = threadIdx.x & 63;
    const int64_t p0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
    if (p0 >= N) return;                               // whole wavefront
    const int64_t pid = p0 + lane;
    const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
    // offsets are clamped to [0, P] so that malformed input cannot read past tri_idx
    const int64_t q_end = min(max(off[plast], (int64_t)0), P);
    const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
    const int64_t my_end = pid < N ? min(max(off[pid + 1], my_off), q_end) : q_end;
    const int64_t q_begin = __shfl(my_off, 0);
    double accI = 0.0, accX = 0.0, accY = 0.0;
    for (int64_t base = q_begin; base < q_end; base += 64) {
        const int64_t q = base + lane;
        const int64_t qq = q < q_end ? q : q_end - 1;
        // owner lane: largest l with my_off(l) <= qq (uniform 6-step search)
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
            if (lo + step < 64 && om <= qq) lo += step;
        }
        const int owner = lo;
        const int64_t ip = p0 + owner < N ? p0 + owner : N - 1;
        double vI = 0.0, vX = 0.0, vY = 0.0;
        if (q < q_end) {
            const int32_t t = tri_idx[q];
            if (t >= 0 && t < T)    // out-of-range triangle indices contribute nothing
                pair_fwd<DEG, ORDER>(K, px[ip], py[ip], invh, rec + (int64_t)t * kRecDoubles, vI, vX, vY);
            if (per_pair) {
                per_pair[q] = vI;
                per_pair[P + q] = vX;
                per_pair[2 * P + q] = vY;
            }
        }
        // segmented inclusive scan over lanes (segments = owners, contiguous)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double uI = __shfl_up(vI, d), uX = __shfl_up(vX, d), uY = __shfl_up(vY, d);
            const int uo = __shfl_up(owner, d);
            if (lane >= d && uo == owner) {
                vI += uI;
                vX += uX;
                vY += uY;
            }
        }
        // particle lane picks its segment's last lane in this round
        const int64_t s0 = my_off > base ? my_off : base;
        const int64_t s1 = my_end < base + 64 ? my_end : base + 64;
        const int src = s1 > s0 ? (int)(s1 - 1 - base) : 0;
        const double rI = __shfl(vI, src), rX = __shfl(vX, src), rY = __shfl(vY, src);
        if (s1 > s0) {
            accI += rI;
            accX += rX;
            accY += rY;
        }
    }
    if (pid < N) {
        I[pid] = accI;
        Gx[pid] = accX;
        Gy[pid] = accY;
    }
}

template <int DEG, int ORDER>
void launch_fwd_t(const KArgs &K, double invh, int64_t N, const double *px, const double *py, const int64_t *off,
                  const int32_t *tri_idx, const double *rec, double *I, double *Gx, double *Gy, double *per_pair,
                  int64_t P, int64_t T, hipStream_t s) {
    const int64_t waves = (N + 63) / 64;
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL((forward_kernel<DEG, ORDER>), dim3((unsigned)blocks), dim3(256), 0, s, K, invh, N, px, py,
                       off, tri_idx, rec, I, Gx, Gy, per_pair, P, T);
}

template <int ORDER>
void launch_fwd_deg(int deg, const KArgs &K, double invh, int64_t N, const double *px, const double *py,
                    const int64_t *off, const int32_t *tri_idx, const double *rec, double *I, double *Gx,
                    double *Gy, double *per_pair, int64_t P, int64_t T, hipStream_t s) {
    if (deg <= 3) launch_fwd_t<3, ORDER>(K, invh, N, px, py, off, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
    else if (deg <= 5) launch_fwd_t<5, ORDER>(K, invh, N, px, py, off, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
    else if (deg <= 8) launch_fwd_t<8, ORDER>(K, invh, N, px, py, off, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
    else launch_fwd_t<11, ORDER>(K, invh, N, px, py, off, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
}

}  // namespace

int launch_prepare(int order, int64_t T, const double *tri, const double *nodal, double h, double *rec,
                   hipStream_t s) {
    if (T == 0) return SPHBI_OK;
    const unsigned blocks = (unsigned)((T + 255) / 256);
    const double invh = 1.0 / h;
    if (order == 0) hipLaunchKernelGGL(prepare_kernel<0>, dim3(blocks), dim3(256), 0, s, T, tri, nodal, invh, rec);
    else if (order == 1) hipLaunchKernelGGL(prepare_kernel<1>, dim3(blocks), dim3(256), 0, s, T, tri, nodal, invh, rec);
    else hipLaunchKernelGGL(prepare_kernel<3>, dim3(blocks), dim3(256), 0, s, T, tri, nodal, invh, rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("prepare launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int launch_forward(int order, int deg, int precision, double tau_edge, const KArgs &K, double h, int64_t N,
                   const double *px, const double *py, const int64_t *offsets, const int32_t *tri_idx, int64_t P,
                   int64_t T, const double *rec, double *I, double *Gx, double *Gy, double *per_pair, hipStream_t s) {
    (void)tau_edge;
    if (precision != SPHBI_FP64) { set_error("precision mode %d not available", precision); return SPHBI_EUNSUPPORTED; }
    if (N == 0) return SPHBI_OK;
    const double invh = 1.0 / h;
    if (order == 0) launch_fwd_deg<0>(deg, K, invh, N, px, py, offsets, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
    else if (order == 1) launch_fwd_deg<1>(deg, K, invh, N, px, py, offsets, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
    else launch_fwd_deg<3>(deg, K, invh, N, px, py, offsets, tri_idx, rec, I, Gx, Gy, per_pair, P, T, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("forward launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
