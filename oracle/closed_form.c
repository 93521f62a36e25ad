/*
 * oracle/closed_form.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The paper's own route to the same integrals, in plain FP64: the
 * decomposition of Sec. 4 (disc, sector, segment and stub pieces, the wedge
 * of Alg. 5, the two- and three-vertex cases T2/T3 and the dispatch of
 * Sec. 4.6) and the closed forms of Sec. 5 (cone formulas, Chebyshev
 * expansions of the segment and stub angular terms, the radial 2F1 term).
 * Only tests, the smoke check and the CPU baseline may load it; it shares
 * no source with the device library.  It is checked against the definition
 * oracle (definition.c) and against closed-form pins.
 *
 * Every piece produces the moment table
 *     Mc[K][n] = int int r^K cos(n theta) dr dtheta,
 *     Ms[K][n] = int int r^K sin(n theta) dr dtheta        (Sec. 3, g_k terms)
 * over (piece) cut by the unit disc, in the particle frame.  A piece is
 * evaluated in a canonical frame theta = alpha + s*theta' (rotation plus
 * optional mirror, eq. improper) and its harmonics are rotated back.
 *
 * Readings of passages that are garbled or silent (all documented):
 *  - sector of Alg. 2 is the counter-clockwise arc sigma1 -> sigma2; spans
 *    above pi are taken as full disc minus the complementary sector;
 *  - segment of eq. segment is D cut by {x >= d} with angular bounds
 *    +-acos(d/r) for r in [d, 1]; d < 0 is the full disc minus the mirrored
 *    segment of |d|;
 *  - stub formula (Sec. 4.3) needs the angle at the near vertex >= pi/2,
 *    otherwise the stub is split at the foot of the perpendicular;
 *    atan2 is atan2(y, x) everywhere;
 *  - wedge (Alg. 5): triangle made counter-clockwise; pieces weighted by
 *    the sign of their signed area (eq. intermediateWedge); no edge hit ->
 *    full disc if the particle is inside, else 0; the third-edge cap is
 *    subtracted;
 *  - T2 = W(v0, vx, v2) - W(v1, vx, v2) with vx on the extension of v0v1;
 *  - radial term int r^a (1 - p^2/r^2)^(m/2) dr: its 2F1 power series in
 *    w = (p/r)^2 (the binomial series integrated term by term) for w <= 1/4,
 *    otherwise closed forms of the m = +-1 family reached through the
 *    contiguous (three-term) relations, with exact base cases.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CF_PI 3.14159265358979323846
#define KM 17   /* radial powers K = 0..16 */
#define NM 6    /* harmonics n = 0..5 */

/* moment table; only K < km and n < nm are formed (km = kernel degree +
 * field order + 2 and nm = field order + 2 are all that the contraction
 * reads) */
typedef struct { int km, nm; double c[KM][NM], s[KM][NM]; } mom;

/* an empty table with the limits of `like` */
static void mom_init(mom *C, const mom *like) {
    const int km = like->km, nm = like->nm;     /* like may be C itself */
    memset(C, 0, sizeof(*C));
    C->km = km;
    C->nm = nm;
}

/* kernel description shared with definition.c (same library) */
typedef struct {
    int npieces;
    double R[2];
    int a[2];
    int ng[2];
    double g[2][4];
    double Cd;
} okern;
int oracle_kernel(int id, okern *K);
int oracle_kernel_monomials(int id, int *npieces, double *R, int *deg, double *b, double *Cd);

/* ------------------------------------------------------------------ */
/* Chebyshev coefficients (Sec. 5.1): T_n(x) = sum_j tn[n][j] x^j,      */
/* U_n(x) = sum_j un[n][j] x^j, built by the three-term recurrences.    */
/* ------------------------------------------------------------------ */
static double tn[NM + 1][NM + 1], un[NM + 1][NM + 1];
static int cheb_ready = 0;

static void cheb_init(void) {
    if (cheb_ready) return;
#pragma omp critical(cf_cheb_init)
    {
        if (!cheb_ready) {
            memset(tn, 0, sizeof(tn));
            memset(un, 0, sizeof(un));
            tn[0][0] = 1; tn[1][1] = 1;
            un[0][0] = 1; un[1][1] = 2;
            for (int n = 2; n <= NM; ++n)
                for (int j = 0; j <= NM; ++j) {
                    tn[n][j] = (j ? 2 * tn[n - 1][j - 1] : 0) - tn[n - 2][j];
                    un[n][j] = (j ? 2 * un[n - 1][j - 1] : 0) - un[n - 2][j];
                }
            cheb_ready = 1;
        }
    }
}

/* ------------------------------------------------------------------ */
/* radial term J(a, m) = int_{r0}^{r1} r^a (1 - p^2/r^2)^{m/2} dr        */
/* (Sec. 5.1, the "square root" integral), p <= r0 <= r1.               */
/* ------------------------------------------------------------------ */
static double pw(double r, int e) {           /* r^e for integer e */
    double v = 1.0;
    int k = e < 0 ? -e : e;
    double b = r;
    while (k) { if (k & 1) v *= b; b *= b; k >>= 1; }
    return e < 0 ? 1.0 / v : v;
}

static double P_int(int e, double r0, double r1) {   /* int r^e dr */
    if (e == -1) return log(r1 / r0);
    return (pw(r1, e + 1) - pw(r0, e + 1)) / (e + 1);
}

/* antiderivative of r^c / sqrt(r^2 - p^2) (base cases and the contiguous
 * recurrence c Phi_c = r^{c-1} w + (c-1) p^2 Phi_{c-2}); w = sqrt(r^2 - p^2)
 * is passed in, computed from the geometry (distance along the line from
 * the foot of the perpendicular), because forming it from r and p loses
 * half the digits when r is close to p. */
static double Phi(int c, double r, double w, double p) {
    if (c == 0) return log((r + w) / p);
    if (c == 1) return w;
    if (c == -1) return atan2(w, p) / p;
    if (c == -2) return w / (p * p * r);
    if (c >= 2) return (pw(r, c - 1) * w + (c - 1) * p * p * Phi(c - 2, r, w, p)) / c;
    /* c <= -3: (c+2) Phi_{c+2} = r^{c+1} w + (c+1) p^2 Phi_c */
    return ((c + 2) * Phi(c + 2, r, w, p) - pw(r, c + 1) * w) / ((c + 1) * p * p);
}

static double binom_int(int n, int k) {
    double v = 1.0;
    for (int i = 0; i < k; ++i) v = v * (n - i) / (i + 1);
    return v;
}

/* J(a, m) with w0 = sqrt(r0^2 - p^2), w1 = sqrt(r1^2 - p^2) supplied */
static double radial(int a, int m, double p, double r0, double w0, double r1, double w1) {
    if (!(r1 > r0)) return 0.0;
    if (p <= 0.0) return P_int(a, r0, r1);
    if (m >= 0 && (m % 2) == 0) {                 /* terminating: (1 - w)^{m/2} polynomial */
        double s = 0.0;
        for (int i = 0; i <= m / 2; ++i)
            s += binom_int(m / 2, i) * pw(-p * p, i) * P_int(a - 2 * i, r0, r1);
        return s;
    }
    double q0 = (p / r0) * (p / r0);
    if (q0 <= 0.25) {
        /* 2F1 power series in (p/r)^2: sum_k (-1)^k binom(m/2, k) p^{2k} int r^{a-2k} dr */
        double nu = 0.5 * m, cb = 1.0, s = 0.0, p2k = 1.0;
        for (int k = 0; k < 200; ++k) {
            double t = cb * p2k * P_int(a - 2 * k, r0, r1);
            s += t;
            if (k > 2 && fabs(t) <= 1e-18 * fabs(s)) break;
            cb *= -(nu - k) / (k + 1);
            p2k *= p * p;
        }
        return s;
    }
    /* odd m = 2 mu + 1: (1-p^2/r^2)^{mu+1} (1-p^2/r^2)^{-1/2} */
    int mu1 = (m + 1) / 2;
    double s = 0.0;
    for (int i = 0; i <= mu1; ++i) {
        int c = a - 2 * i + 1;
        s += binom_int(mu1, i) * pw(-p * p, i) * (Phi(c, r1, w1, p) - Phi(c, r0, w0, p));
    }
    return s;
}

double oracle_cf_radial(int a, int m, double p, double r0, double r1) {
    double w0 = sqrt(fmax(r0 * r0 - p * p, 0.0)), w1 = sqrt(fmax(r1 * r1 - p * p, 0.0));
    return radial(a, m, p, r0, w0, r1, w1);
}

/* ------------------------------------------------------------------ */
/* canonical pieces                                                     */
/* ------------------------------------------------------------------ */

/* rotate canonical moments back: theta = alpha + s theta' (eq. improper) */
static void add_rotated(mom *M, const mom *C, double alpha, int s, double sign) {
    for (int n = 0; n < C->nm; ++n) {
        double cn = cos(n * alpha), sn = sin(n * alpha);
        for (int K = 0; K < C->km; ++K) {
            double c = C->c[K][n], si = C->s[K][n];
            M->c[K][n] += sign * (cn * c - s * sn * si);
            M->s[K][n] += sign * (sn * c + s * cn * si);
        }
    }
}

/* Alg. 1: full disc of radius 1 */
static void disc(mom *C) {
    mom_init(C, C);
    for (int K = 0; K < C->km; ++K) C->c[K][0] = 2.0 * CF_PI / (K + 1);
}

/* cone closed forms (Sec. 5.2): sector theta' in [0, g], r in [0, d] */
static void sector_c(mom *C, double g, double d) {
    mom_init(C, C);
    for (int K = 0; K < C->km; ++K) {
        double rad = pw(d, K + 1) / (K + 1);
        C->c[K][0] = g * rad;
        for (int n = 1; n < C->nm; ++n) {
            C->c[K][n] = rad * sin(n * g) / n;
            C->s[K][n] = rad * (1.0 - cos(n * g)) / n;
        }
    }
}

/* segment closed forms (Sec. 5.3), d >= 0: r in [d,1], |theta'| <= acos(d/r) */
static void segment_c(mom *C, double d) {
    mom_init(C, C);
    if (d >= 1.0) return;
    double w1 = sqrt((1.0 - d) * (1.0 + d));          /* half chord */
    double ac = atan2(w1, d);                          /* acos(d) */
    for (int K = 1; K < C->km; ++K) {
        /* n = 0: 2 int r^K acos(d/r) = 2 [r^{K+1} acos(d/r)/(K+1)] - 2 d/(K+1) J(K-1,-1) */
        double v = ac / (K + 1);
        if (d > 0) v -= d / (K + 1) * radial(K - 1, -1, d, d, 0.0, 1.0, w1);
        C->c[K][0] = 2.0 * v;
        for (int n = 1; n < C->nm; ++n) {
            /* (2/n) sum_j u_{n-1,j} d^j J(K-j, 1) */
            double s = 0.0;
            for (int j = 0; j < n; ++j) {
                if (un[n - 1][j] == 0.0) continue;
                if (d == 0.0 && j > 0) continue;
                s += un[n - 1][j] * pw(d, j) * radial(K - j, 1, d, d, 0.0, 1.0, w1);
            }
            C->c[K][n] = 2.0 * s / n;
        }
    }
}

/* D cut by the half plane {x . (cos a, sin a) >= dd} */
static void segment_piece(mom *M, double a, double dd, double sign) {
    mom C;
    mom_init(&C, M);
    if (dd >= 1.0) return;
    if (dd <= -1.0) { disc(&C); add_rotated(M, &C, 0.0, 1, sign); return; }
    if (dd >= 0.0) {
        segment_c(&C, dd);
    } else {
        mom S;
        mom_init(&S, M);
        segment_c(&S, -dd);
        disc(&C);
        for (int K = 0; K < C.km; ++K)
            for (int n = 0; n < C.nm; ++n) C.c[K][n] -= ((n & 1) ? -1.0 : 1.0) * S.c[K][n];
    }
    add_rotated(M, &C, a, 1, sign);
}

static double cross2(const double *a, const double *b) { return a[0] * b[1] - a[1] * b[0]; }
static double dot2(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1]; }
static double norm2(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1]); }
static double sgn(double x) { return (x > 0) - (x < 0); }

/* Alg. 2: sector from the direction of v1 counter-clockwise to v2 (< pi) */
static void sector_piece(mom *M, const double *v1, const double *v2, double sign) {
    double a1 = atan2(v1[1], v1[0]);
    double x = cos(-a1) * v2[0] - sin(-a1) * v2[1];
    double y = sin(-a1) * v2[0] + cos(-a1) * v2[1];
    int s = y >= 0 ? 1 : -1;
    double g = atan2(s * y, x);
    mom C;
    mom_init(&C, M);
    sector_c(&C, g, 1.0);
    add_rotated(M, &C, a1, s, sign);
}

/* Sec. 4.3 / Alg. 4 integrateR: stub (0, near, far) whose angle at the near
 * vertex is >= pi/2, cut by the unit disc.  The stub is described by the
 * distance p of its far edge's line from the particle and the distances
 * wn <= wf of the near and far vertex from the foot of the perpendicular,
 * so that |near| = sqrt(p^2 + wn^2), |far| = sqrt(p^2 + wf^2),
 * asin(p/r) = atan2(p, w) and beta = atan2(p, wf) (angle at the far
 * vertex); alpha/s place the far vertex on the canonical x axis with the
 * near vertex above it. */
static void integrateR(mom *M, double p, double wn, double wf, double alpha, int s, double sign) {
    double d = sqrt(p * p + wn * wn), l = sqrt(p * p + wf * wf);
    double gam = atan2(wf, p) - atan2(wn, p);              /* angle at the origin */
    if (!(gam > 0.0) || l == 0.0) return;
    double beta = atan2(p, wf);                             /* angle at the far vertex */
    mom C;
    mom_init(&C, M);
    sector_c(&C, gam, fmin(d, 1.0));                        /* S(gamma, |nu_near|) */
    if (d < 1.0) {
        double r1 = l, w1 = wf;
        if (l > 1.0) { r1 = 1.0; w1 = sqrt((1.0 - p) * (1.0 + p)); }
        double cb[NM], sb[NM];
        for (int n = 0; n < C.nm; ++n) { cb[n] = cos(n * beta); sb[n] = sin(n * beta); }
        double as1 = atan2(p, w1), as0 = atan2(p, wn);      /* asin(p/r) at both ends */
        for (int K = 1; K < C.km; ++K) {
            double PK = P_int(K, d, r1);
            /* n = 0: int r^K (asin(p/r) - beta) dr */
            double v = (pw(r1, K + 1) * as1 - pw(d, K + 1) * as0) / (K + 1);
            if (p > 0) v += p / (K + 1) * radial(K - 1, -1, p, d, wn, r1, w1);
            C.c[K][0] += v - beta * PK;
            for (int n = 1; n < C.nm; ++n) {
                /* sin(n asin s) = s U_{n-1}(c), cos(n asin s) = T_n(c), c = sqrt(1 - s^2) */
                double SU = 0.0, CT = 0.0;
                if (p > 0)
                    for (int j = 0; j < n; ++j)
                        if (un[n - 1][j] != 0.0) SU += un[n - 1][j] * radial(K - 1, j, p, d, wn, r1, w1);
                SU *= p;
                for (int j = 0; j <= n; ++j)
                    if (tn[n][j] != 0.0) CT += tn[n][j] * radial(K, j, p, d, wn, r1, w1);
                /* sin(n omega) = sin(n asin s) cos(n beta) - cos(n asin s) sin(n beta) */
                C.c[K][n] += (cb[n] * SU - sb[n] * CT) / n;
                /* 1 - cos(n omega), cos(n omega) = cos(n asin s) cos(n beta) + sin(n asin s) sin(n beta) */
                C.s[K][n] += (PK - cb[n] * CT - sb[n] * SU) / n;
            }
        }
    }
    add_rotated(M, &C, alpha, s, sign);
}

/* Alg. 4 triangularIntegral: stub (0, a, b) cut by the disc, split at the
 * foot of the perpendicular when the angle at the near vertex is < pi/2. */
static void stub(mom *M, const double *a, const double *b, double sign) {
    double e[2] = {b[0] - a[0], b[1] - a[1]};
    double L = norm2(e);
    if (L == 0.0) return;
    double u[2] = {e[0] / L, e[1] / L};
    double ya = dot2(a, u), yb = ya + L;                    /* positions along the line */
    double cr = cross2(a, u);                               /* signed distance of the line */
    double p = fabs(cr);
    if (p == 0.0) return;
    /* canonical frame of a sub-stub: far vertex on the x axis, near vertex above */
    if (ya < 0.0 && yb > 0.0) {                            /* foot inside: split at nu_c */
        double fa = atan2(a[1], a[0]), fb = atan2(b[1], b[0]);
        /* sub-stubs (c, a) and (c, b): cross(a, c) = -ya cr, cross(b, c) = -yb cr */
        integrateR(M, p, 0.0, -ya, fa, cr > 0 ? 1 : -1, sign);
        integrateR(M, p, 0.0, yb, fb, cr > 0 ? -1 : 1, sign);
    } else {
        int a_near = fabs(ya) <= fabs(yb);
        const double *fr = a_near ? b : a;
        double wn = a_near ? fabs(ya) : fabs(yb), wf = a_near ? fabs(yb) : fabs(ya);
        double f = atan2(fr[1], fr[0]);
        /* near above the far ray: sign of cross(far, near) */
        double c = a_near ? cross2(b, a) : cross2(a, b);
        integrateR(M, p, wn, wf, f, c >= 0 ? 1 : -1, sign);
    }
}

static double seg_dist(const double *a, const double *b) {   /* distance of 0 to segment ab */
    double e[2] = {b[0] - a[0], b[1] - a[1]};
    double L2 = dot2(e, e);
    double t = L2 > 0 ? -dot2(a, e) / L2 : 0.0;
    t = t < 0 ? 0 : (t > 1 ? 1 : t);
    double q[2] = {a[0] + t * e[0], a[1] + t * e[1]};
    return norm2(q);
}

/* line-circle intersection (lci of Alg. 3): largest lambda with |o + lambda d| = 1 */
static double lci_far(const double *o, const double *d) {
    double A = dot2(d, d), B = 2.0 * dot2(o, d), Cc = dot2(o, o) - 1.0;
    double disc = B * B - 4.0 * A * Cc;
    if (disc < 0) disc = 0;
    double sq = sqrt(disc);
    /* stable roots */
    double q = -0.5 * (B + (B >= 0 ? sq : -sq));
    double l1 = q / A, l2 = (q != 0.0) ? Cc / q : l1;
    return l1 > l2 ? l1 : l2;
}

/* half plane D cut by line ab on the side away from / toward point c */
static void half_plane_piece(mom *M, const double *a, const double *b, const double *c, int toward,
                             double sign) {
    double e[2] = {b[0] - a[0], b[1] - a[1]};
    double L = norm2(e);
    double nrm[2] = {-e[1] / L, e[0] / L};
    double side = dot2(nrm, c) - dot2(nrm, a);
    if ((side < 0) == (toward != 0)) { nrm[0] = -nrm[0]; nrm[1] = -nrm[1]; }
    segment_piece(M, atan2(nrm[1], nrm[0]), dot2(nrm, a), sign);
}

/* Alg. 5: triangle with at most one vertex inside the unit disc */
static void wedge(mom *M, const double *V0, const double *V1, const double *V2, double sign) {
    double v[3][2] = {{V0[0], V0[1]}, {V1[0], V1[1]}, {V2[0], V2[1]}};
    double ar = (v[1][0] - v[0][0]) * (v[2][1] - v[0][1]) - (v[2][0] - v[0][0]) * (v[1][1] - v[0][1]);
    if (ar == 0.0) return;
    if (ar < 0) {                               /* counter-clockwise, as Sec. 4.4 asks */
        double t0 = v[1][0], t1 = v[1][1];
        v[1][0] = v[2][0]; v[1][1] = v[2][1]; v[2][0] = t0; v[2][1] = t1;
    }
    int hit[3];
    int nh = 0;
    for (int e = 0; e < 3; ++e) { hit[e] = seg_dist(v[e], v[(e + 1) % 3]) < 1.0; nh += hit[e]; }
    if (nh == 0) {
        int in = 1;
        for (int e = 0; e < 3; ++e) {
            double a[2] = {v[(e + 1) % 3][0] - v[e][0], v[(e + 1) % 3][1] - v[e][1]};
            double o[2] = {-v[e][0], -v[e][1]};
            if (cross2(a, o) < 0) in = 0;
        }
        if (in) { mom C; mom_init(&C, M); disc(&C); add_rotated(M, &C, 0.0, 1, sign); }
        return;
    }
    if (nh == 1) {
        int e = hit[0] ? 0 : (hit[1] ? 1 : 2);
        half_plane_piece(M, v[e], v[(e + 1) % 3], v[(e + 2) % 3], 1, sign);
        return;
    }
    /* apex: the inside vertex, else the vertex shared by two hit edges */
    int apex = -1;
    for (int i = 0; i < 3; ++i) if (dot2(v[i], v[i]) <= 1.0) apex = i;
    if (apex < 0) {
        if (nh == 3 || (hit[2] && hit[0])) apex = 0;
        else if (hit[0] && hit[1]) apex = 1;
        else apex = 2;
    }
    const double *a0 = v[apex], *a1 = v[(apex + 1) % 3], *a2 = v[(apex + 2) % 3];
    double d1[2] = {a1[0] - a0[0], a1[1] - a0[1]}, d2[2] = {a2[0] - a0[0], a2[1] - a0[1]};
    double l1 = lci_far(a0, d1), l2 = lci_far(a0, d2);
    double s1[2] = {a0[0] + l1 * d1[0], a0[1] + l1 * d1[1]};
    double s2[2] = {a0[0] + l2 * d2[0], a0[1] + l2 * d2[1]};
    /* eq. intermediateWedge: sign-weighted stubs and the arc */
    double sa = sgn(cross2(a0, s1)), sb = sgn(cross2(s2, a0));
    if (sa != 0) stub(M, a0, s1, sign * sa);
    if (sb != 0) stub(M, s2, a0, sign * sb);
    double span = atan2(cross2(s1, s2), dot2(s1, s2));     /* (-pi, pi] */
    if (span >= 0) {
        sector_piece(M, s1, s2, sign);
    } else {                                                /* arc longer than pi */
        mom C;
        mom_init(&C, M);
        disc(&C);
        add_rotated(M, &C, 0.0, 1, sign);
        sector_piece(M, s2, s1, -sign);
    }
    /* third edge crossing: remove the cap beyond it (away from the apex) */
    int e3 = (apex + 1) % 3;
    if (hit[e3]) half_plane_piece(M, a1, a2, a0, 0, -sign);
}

/* Sec. 4.5-4.6: dispatch on the number of vertices inside */
static void triangle_moments(mom *M, double v[3][2]) {
    int in[3], ni = 0;
    for (int i = 0; i < 3; ++i) { in[i] = (v[i][0] * v[i][0] + v[i][1] * v[i][1]) <= 1.0; ni += in[i]; }
    if (ni <= 1) {
        int a = in[1] ? 1 : (in[2] ? 2 : 0);
        wedge(M, v[a], v[(a + 1) % 3], v[(a + 2) % 3], 1.0);
        return;
    }
    if (ni == 2) {
        int o = !in[0] ? 0 : (!in[1] ? 1 : 2);              /* the outside vertex */
        const double *p0 = v[(o + 1) % 3], *p1 = v[(o + 2) % 3], *p2 = v[o];
        double e[2] = {p1[0] - p0[0], p1[1] - p0[1]};
        double L = norm2(e);
        if (L == 0.0) return;
        double vx[2] = {p0[0] + 3.0 * e[0] / L, p0[1] + 3.0 * e[1] / L};
        wedge(M, p0, vx, p2, 1.0);                          /* T2 = W(v0,vx,v2) - W(v1,vx,v2) */
        wedge(M, p1, vx, p2, -1.0);
        return;
    }
    /* T3 = W(v0, x1, x2) - T2(v1, x1, v2) - W(v2, x1, x2) */
    double e1[2] = {v[1][0] - v[0][0], v[1][1] - v[0][1]}, e2[2] = {v[2][0] - v[0][0], v[2][1] - v[0][1]};
    double L1 = norm2(e1), L2 = norm2(e2);
    if (L1 == 0.0 || L2 == 0.0) return;
    double x1[2] = {v[0][0] + 3.0 * e1[0] / L1, v[0][1] + 3.0 * e1[1] / L1};
    double x2[2] = {v[0][0] + 3.0 * e2[0] / L2, v[0][1] + 3.0 * e2[1] / L2};
    wedge(M, v[0], x1, x2, 1.0);
    {   /* T2 on (v1, v2 inside; x1 outside): W(v1, y, x1) - W(v2, y, x1), y beyond v2 on v1v2 */
        double e[2] = {v[2][0] - v[1][0], v[2][1] - v[1][1]};
        double L = norm2(e);
        if (L > 0.0) {
            double y[2] = {v[1][0] + 3.0 * e[0] / L, v[1][1] + 3.0 * e[1] / L};
            wedge(M, v[1], y, x1, -1.0);
            wedge(M, v[2], y, x1, 1.0);
        }
    }
    wedge(M, v[2], x1, x2, -1.0);
}

/* ------------------------------------------------------------------ */
/* field polynomial about the particle (Sec. 3) and contraction         */
/* ------------------------------------------------------------------ */
typedef struct { double c[4][4]; } bpoly;   /* c[i][j] x^i y^j, i + j <= 3 */

static void bp_mul(bpoly *r, const bpoly *a, const bpoly *b) {
    bpoly t;
    memset(&t, 0, sizeof(t));
    for (int i = 0; i < 4; ++i)
        for (int j = 0; i + j < 4; ++j)
            for (int k = 0; i + k < 4; ++k)
                for (int l = 0; j + l < 4 && i + j + k + l < 4; ++l) t.c[i + k][j + l] += a->c[i][j] * b->c[k][l];
    *r = t;
}

static void field_poly(int nn, double v[3][2], const double *A, bpoly *F) {
    memset(F, 0, sizeof(*F));
    if (nn == 1) { F->c[0][0] = A[0]; return; }
    double x0 = v[0][0], y0 = v[0][1], x1 = v[1][0], y1 = v[1][1], x2 = v[2][0], y2 = v[2][1];
    double D = (y1 - y2) * (x0 - x2) + (x2 - x1) * (y0 - y2);
    if (nn == 3) {                                   /* eq. taus */
        double L0 = (y1 - y2) * (A[0] - A[2]) / D, L1 = (x2 - x1) * (A[0] - A[2]) / D;
        double L2 = (y2 - y0) * (A[1] - A[2]) / D, L3 = (x0 - x2) * (A[1] - A[2]) / D;
        double t1 = L0 + L2, t2 = L1 + L3;
        F->c[1][0] = t1;
        F->c[0][1] = t2;
        F->c[0][0] = A[2] - (L0 * x2 + L1 * y2 + L2 * x2 + L3 * y2);
        return;
    }
    /* cubic Lagrange: lambda_i affine in (x, y); expand the basis products */
    bpoly l[3];
    memset(l, 0, sizeof(l));
    l[0].c[0][0] = ((y1 - y2) * (-x2) + (x2 - x1) * (-y2)) / D;
    l[0].c[1][0] = (y1 - y2) / D;
    l[0].c[0][1] = (x2 - x1) / D;
    l[1].c[0][0] = ((y2 - y0) * (-x2) + (x0 - x2) * (-y2)) / D;
    l[1].c[1][0] = (y2 - y0) / D;
    l[1].c[0][1] = (x0 - x2) / D;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) l[2].c[i][j] = -l[0].c[i][j] - l[1].c[i][j];
    l[2].c[0][0] += 1.0;
    bpoly m3[3], m1[3];                               /* 3 lambda - 1, 3 lambda - 2 */
    for (int i = 0; i < 3; ++i) {
        m3[i] = l[i];
        for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) m3[i].c[a][b] *= 3.0;
        m1[i] = m3[i];
        m3[i].c[0][0] -= 1.0;
        m1[i].c[0][0] -= 2.0;
    }
    bpoly t, u;
    for (int i = 0; i < 3; ++i) {                    /* vertices: lambda (3 lambda-1)(3 lambda-2)/2 */
        bp_mul(&t, &l[i], &m3[i]);
        bp_mul(&u, &t, &m1[i]);
        for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) F->c[a][b] += 0.5 * A[i] * u.c[a][b];
    }
    static const int ea[3] = {0, 1, 2}, eb[3] = {1, 2, 0};
    for (int e = 0; e < 3; ++e) {
        bpoly ll;
        bp_mul(&ll, &l[ea[e]], &l[eb[e]]);
        bp_mul(&u, &ll, &m3[ea[e]]);
        for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) F->c[a][b] += 4.5 * A[3 + 2 * e] * u.c[a][b];
        bp_mul(&u, &ll, &m3[eb[e]]);
        for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) F->c[a][b] += 4.5 * A[4 + 2 * e] * u.c[a][b];
    }
    bp_mul(&t, &l[0], &l[1]);
    bp_mul(&u, &t, &l[2]);
    for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) F->c[a][b] += 27.0 * A[9] * u.c[a][b];
}

/* cos^i sin^j (times cos, sin or 1) as a sum of harmonics (product-to-sum) */
typedef struct { double c[NM], s[NM]; } trig;

static void trig_mul_cs(trig *t, int by_sin) {
    trig r;
    memset(&r, 0, sizeof(r));
    for (int n = 0; n < NM - 1; ++n) {
        double c = t->c[n], s = t->s[n];
        if (c == 0.0 && s == 0.0) continue;
        int m = n - 1;
        if (!by_sin) {     /* cos n cos = (cos(n+1) + cos(n-1))/2 ; sin n cos = (sin(n+1) + sin(n-1))/2 */
            r.c[n + 1] += 0.5 * c;
            r.s[n + 1] += 0.5 * s;
            if (m >= 0) { r.c[m] += 0.5 * c; r.s[m] += 0.5 * s; }
            else { r.c[1] += 0.5 * c; r.s[1] -= 0.5 * s; }
        } else {           /* cos n sin = (sin(n+1) - sin(n-1))/2 ; sin n sin = (cos(n-1) - cos(n+1))/2 */
            r.s[n + 1] += 0.5 * c;
            r.c[n + 1] -= 0.5 * s;
            if (m >= 0) { r.s[m] -= 0.5 * c; r.c[m] += 0.5 * s; }
            else { r.s[1] += 0.5 * c; r.c[1] += 0.5 * s; }
        }
    }
    *t = r;
}

static void trig_monomial(int i, int j, int extra, trig *t) {   /* extra: 0 none, 1 cos, 2 sin */
    memset(t, 0, sizeof(*t));
    t->c[0] = 1.0;
    for (int a = 0; a < i; ++a) trig_mul_cs(t, 0);
    for (int b = 0; b < j; ++b) trig_mul_cs(t, 1);
    if (extra == 1) trig_mul_cs(t, 0);
    if (extra == 2) trig_mul_cs(t, 1);
}

static double contract(const mom *M, int K, const trig *t) {
    double s = 0.0;
    if (K < 0 || K >= M->km) return 0.0;
    for (int n = 0; n < M->nm; ++n) s += t->c[n] * M->c[K][n] + t->s[n] * M->s[K][n];
    return s;
}

static void cf_pair_normalised(int kid, int nn, double v[3][2], const double *A, double out[3]) {
    cheb_init();
    int np, deg[2];
    double R[2], b[24], Cd;
    oracle_kernel_monomials(kid, &np, R, deg, b, &Cd);
    out[0] = out[1] = out[2] = 0.0;
    double ar = (v[1][0] - v[0][0]) * (v[2][1] - v[0][1]) - (v[2][0] - v[0][0]) * (v[1][1] - v[0][1]);
    if (ar == 0.0 || !isfinite(ar)) return;
    bpoly F;
    field_poly(nn, v, A, &F);
    for (int p = 0; p < np; ++p) {
        double s[3][2];
        for (int i = 0; i < 3; ++i) { s[i][0] = v[i][0] / R[p]; s[i][1] = v[i][1] / R[p]; }
        mom M;
        memset(&M, 0, sizeof(M));
        {
            const int order = nn == 1 ? 0 : (nn == 3 ? 1 : 3);
            M.km = deg[p] + order + 2 < KM ? deg[p] + order + 2 : KM;
            M.nm = order + 2;
        }
        triangle_moments(&M, s);
        for (int K = 0; K < M.km; ++K) {                   /* back to radius R_p */
            double f = pw(R[p], K + 1);
            for (int n = 0; n < M.nm; ++n) { M.c[K][n] *= f; M.s[K][n] *= f; }
        }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; i + j < 4; ++j) {
                double c = F.c[i][j];
                if (c == 0.0) continue;
                trig t0, tx, ty;
                trig_monomial(i, j, 0, &t0);
                trig_monomial(i, j, 1, &tx);
                trig_monomial(i, j, 2, &ty);
                for (int k = 0; k <= deg[p]; ++k) {
                    double bk = b[12 * p + k];
                    if (bk == 0.0) continue;
                    /* value: b_k r^{k} A r dr -> K = k + 1 + i + j */
                    out[0] += bk * c * contract(&M, k + 1 + i + j, &t0);
                    /* gradient (eq. basicdiff, G1): -k b_k r^{k-1} A e r dr -> K = k + i + j */
                    if (k > 0) {
                        out[1] -= k * bk * c * contract(&M, k + i + j, &tx);
                        out[2] -= k * bk * c * contract(&M, k + i + j, &ty);
                    }
                }
            }
    }
    out[0] *= Cd;
    out[1] *= Cd;
    out[2] *= Cd;
}

int oracle_cf_pair(int kid, double h, int nn, double px, double py, const double *tri6, const double *A,
                   double *out) {
    if (!(h > 0) || (nn != 1 && nn != 3 && nn != 10) || kid < 0 || kid > 3) return -1;
    double v[3][2];
    for (int i = 0; i < 3; ++i) {
        v[i][0] = (tri6[2 * i] - px) / h;
        v[i][1] = (tri6[2 * i + 1] - py) / h;
    }
    cf_pair_normalised(kid, nn, v, A, out);
    out[1] /= h;
    out[2] /= h;
    return 0;
}

int oracle_cf_integrate(int kid, double h, int nn, int64_t N, const double *px, const double *py, int64_t T,
                        const double *tri, const double *nodal, const int64_t *offsets, const int32_t *tri_idx,
                        double *I, double *Gx, double *Gy, double *per_pair, int nthreads) {
    if (!(h > 0) || (nn != 1 && nn != 3 && nn != 10) || kid < 0 || kid > 3 || N < 0 || T < 0) return -1;
    cheb_init();
    int64_t P = N > 0 ? offsets[N] : 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|:bad)
    for (int64_t i = 0; i < N; ++i) {
        double si = 0, sx = 0, sy = 0;
        for (int64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
            int64_t j = tri_idx[q];
            if (j < 0 || j >= T) { bad = 1; continue; }
            double v[3][2], A[10], o[3];
            for (int k = 0; k < 3; ++k) {
                v[k][0] = (tri[(2 * k) * T + j] - px[i]) / h;
                v[k][1] = (tri[(2 * k + 1) * T + j] - py[i]) / h;
            }
            for (int a = 0; a < nn; ++a) A[a] = nodal[a * T + j];
            cf_pair_normalised(kid, nn, v, A, o);
            o[1] /= h;
            o[2] /= h;
            if (per_pair) { per_pair[q] = o[0]; per_pair[P + q] = o[1]; per_pair[2 * P + q] = o[2]; }
            si += o[0]; sx += o[1]; sy += o[2];
        }
        I[i] = si; Gx[i] = sx; Gy[i] = sy;
    }
    return bad ? -2 : 0;
}
