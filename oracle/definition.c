/*
 * oracle/definition.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow FP64 evaluation of the SPH boundary integrals straight from
 * their definition.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library; the product path never
 * does.  It shares no source with the device library.
 *
 * For a particle at x, support radius h, kernel W(r) = C_d h^-2 k(r/h) and a
 * triangle T carrying a polynomial field A_T, it computes
 *
 *     I(x) = int_T A_T(x') W(|x - x'|) dx'                     (Sec. 2, eq. sphintegral/boundaryint)
 *     G(x) = int_T A_T(x') grad_x W(|x - x'|) dx'               (Sec. 2, eq. nablaIntegral)
 *
 * in the frame normalised by the transform C of Sec. 2 (particle at the
 * origin, support 1): I = C_d int A k(|xi|) dxi and
 * G = -(C_d/h) int A (xi/|xi|) k'(|xi|) dxi (Sec. 3, eq. basicdiff).
 *
 * Evaluation: polar coordinates about the particle (Sec. 3, eq.
 * singleSpherical).  For every direction theta the ray meets the triangle
 * in one interval [r_in, r_out]; its intersection with each kernel piece
 * r < R_p is integrated EXACTLY by a Gauss-Legendre rule whose degree
 * exceeds the polynomial degree of A(r e_theta) k(r) r (nothing but a
 * polynomial on that interval).  The outer theta integral is split at every
 * vertex direction and every edge/circle crossing -- the only places where
 * the integrand stops being analytic -- and integrated by adaptive
 * bisection with a 10/20-point Gauss-Legendre error estimate.  The kernel is
 * evaluated in its factored form (1 - q/R)^a g(q/R), never in monomials.
 *
 * Fields (Sec. 3): P0 constant, P1 barycentric (eq. for lambda_0, lambda_1),
 * P3 cubic Lagrange on the 10 nodes v0, v1, v2, edge v0v1 at 1/3 and 2/3,
 * edge v1v2 at 1/3, 2/3, edge v2v0 at 1/3, 2/3, centroid (the paper only
 * says that FEM stencils in barycentric coordinates are admissible).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* kernels: k(q) = sum_p [q < R_p] (1 - q/R_p)^a_p g_p(q/R_p)          */
/* ------------------------------------------------------------------ */
typedef struct {
    int npieces;
    double R[2];
    int a[2];
    int ng[2];
    double g[2][4];
    double Cd;
} okern;

/* Gauss-Legendre rules, built once by Newton iteration on P_n. */
#define GL_MAXN 24
static double gl_x[GL_MAXN + 1][GL_MAXN], gl_w[GL_MAXN + 1][GL_MAXN];
static int gl_ready = 0;

static void gl_build(int n) {
    for (int i = 0; i < n; ++i) {
        double x = cos(OR_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (x * p1 - p0) / (x * x - 1.0);
        gl_x[n][i] = x;
        gl_w[n][i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

static void gl_init(void) {
    if (gl_ready) return;
#pragma omp critical(oracle_gl_init)
    {
        if (!gl_ready) {
            for (int n = 1; n <= GL_MAXN; ++n) gl_build(n);
            gl_ready = 1;
        }
    }
}

static double poly_eval(const double *c, int n, double t) {
    double s = 0.0;
    for (int i = n - 1; i >= 0; --i) s = s * t + c[i];
    return s;
}

static double poly_deriv(const double *c, int n, double t) {
    double s = 0.0;
    for (int i = n - 1; i >= 1; --i) s = s * t + i * c[i];
    return s;
}

/* k_p(q) for q < R_p */
static double kpiece(const okern *K, int p, double q) {
    double t = q / K->R[p];
    return pow(1.0 - t, K->a[p]) * poly_eval(K->g[p], K->ng[p], t);
}

/* dk_p/dq for q < R_p */
static double kpiece_d(const okern *K, int p, double q) {
    double t = q / K->R[p];
    double g = poly_eval(K->g[p], K->ng[p], t);
    double gd = poly_deriv(K->g[p], K->ng[p], t);
    int a = K->a[p];
    return pow(1.0 - t, a - 1) * (-a * g + (1.0 - t) * gd) / K->R[p];
}

/* Wendland C2/C4/C6 and the cubic B-spline; ids are those of the C-ABI. */
int oracle_kernel(int id, okern *K) {
    memset(K, 0, sizeof(*K));
    gl_init();
    switch (id) {
    case 0: /* Wendland C2: (1-q)^4 (1+4q) */
        K->npieces = 1; K->R[0] = 1.0; K->a[0] = 4; K->ng[0] = 2;
        K->g[0][0] = 1.0; K->g[0][1] = 4.0;
        break;
    case 1: /* Wendland C4: (1-q)^6 (1+6q+35/3 q^2), the kernel named in Sec. 2 */
        K->npieces = 1; K->R[0] = 1.0; K->a[0] = 6; K->ng[0] = 3;
        K->g[0][0] = 1.0; K->g[0][1] = 6.0; K->g[0][2] = 35.0 / 3.0;
        break;
    case 2: /* Wendland C6: (1-q)^8 (1+8q+25q^2+32q^3) */
        K->npieces = 1; K->R[0] = 1.0; K->a[0] = 8; K->ng[0] = 4;
        K->g[0][0] = 1.0; K->g[0][1] = 8.0; K->g[0][2] = 25.0; K->g[0][3] = 32.0;
        break;
    case 3: /* cubic B-spline (1-q)^3_+ - 4 (1/2-q)^3_+ ; second piece = -1/2 (1-2q)^3 */
        K->npieces = 2;
        K->R[0] = 1.0; K->a[0] = 3; K->ng[0] = 1; K->g[0][0] = 1.0;
        K->R[1] = 0.5; K->a[1] = 3; K->ng[1] = 1; K->g[1][0] = -0.5;
        break;
    default:
        return -1;
    }
    /* C_d makes the kernel integrate to one over the unit disc:
     * C_d = 1 / (2 pi int_0^1 k(q) q dq); the integrand is a polynomial per
     * piece, so a 12-point rule is exact. */
    double s = 0.0;
    for (int p = 0; p < K->npieces; ++p) {
        double R = K->R[p];
        for (int i = 0; i < 12; ++i) {
            double q = 0.5 * R * (gl_x[12][i] + 1.0);
            s += 0.5 * R * gl_w[12][i] * kpiece(K, p, q) * q;
        }
    }
    K->Cd = 1.0 / (2.0 * OR_PI * s);
    return 0;
}

/* Monomial coefficients b_k of every piece in the variable q (q < R_p). */
int oracle_kernel_monomials(int id, int *npieces, double *R, int *deg, double *b /*[2][12]*/, double *Cd) {
    okern K;
    if (oracle_kernel(id, &K)) return -1;
    *npieces = K.npieces;
    *Cd = K.Cd;
    memset(b, 0, sizeof(double) * 24);
    for (int p = 0; p < K.npieces; ++p) {
        /* (1 - t)^a * g(t), t = q / R */
        double c[16] = {0};
        c[0] = 1.0;
        int n = 1;
        for (int i = 0; i < K.a[p]; ++i) {       /* multiply by (1 - t) */
            for (int j = n; j >= 1; --j) c[j] = c[j] - c[j - 1];
            ++n;
        }
        double r[16] = {0};
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < K.ng[p]; ++j) r[i + j] += c[i] * K.g[p][j];
        int d = n + K.ng[p] - 2;
        R[p] = K.R[p];
        deg[p] = d;
        for (int k = 0; k <= d; ++k) b[p * 12 + k] = r[k] / pow(K.R[p], k);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* field on one triangle (normalised frame)                             */
/* ------------------------------------------------------------------ */
typedef struct {
    double x[3], y[3];
    double D;     /* (y1-y2)(x0-x2) + (x2-x1)(y0-y2), Sec. 3 */
    double orient;
    double elen[3], eang[3], eopp[3], ecr[3];   /* per edge: length, direction angles of e and -e, cross(e, a) */
    int nn;
    double A[10];
} otri;

static void bary(const otri *t, double x, double y, double *l0, double *l1, double *l2) {
    *l0 = ((t->y[1] - t->y[2]) * (x - t->x[2]) + (t->x[2] - t->x[1]) * (y - t->y[2])) / t->D;
    *l1 = ((t->y[2] - t->y[0]) * (x - t->x[2]) + (t->x[0] - t->x[2]) * (y - t->y[2])) / t->D;
    *l2 = 1.0 - *l0 - *l1;
}

static double field_at(const otri *t, double x, double y) {
    if (t->nn == 1) return t->A[0];
    double l[3];
    bary(t, x, y, &l[0], &l[1], &l[2]);
    if (t->nn == 3) return l[0] * t->A[0] + l[1] * t->A[1] + l[2] * t->A[2];
    /* cubic Lagrange basis in barycentric coordinates */
    double v = 0.0;
    for (int i = 0; i < 3; ++i) v += t->A[i] * 0.5 * l[i] * (3.0 * l[i] - 1.0) * (3.0 * l[i] - 2.0);
    static const int ea[3] = {0, 1, 2}, eb[3] = {1, 2, 0};
    for (int e = 0; e < 3; ++e) {
        double la = l[ea[e]], lb = l[eb[e]];
        v += t->A[3 + 2 * e] * 4.5 * la * lb * (3.0 * la - 1.0);      /* node at 1/3 from v_a */
        v += t->A[4 + 2 * e] * 4.5 * la * lb * (3.0 * lb - 1.0);      /* node at 2/3 from v_a */
    }
    v += t->A[9] * 27.0 * l[0] * l[1] * l[2];
    return v;
}

/* ------------------------------------------------------------------ */
/* radial integral along one direction                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    const okern *K;
    const otri *t;
    int nr;                 /* radial GL points */
    long calls;
    double tol;
    int capped;             /* an interval was accepted at a cap, not by its error estimate */
} octx;

/* value, and radial part of the gradient (before the -e_theta factor) */
/* Ray at angle theta = base + delta, where base is an end of the current
 * interval and delta the (small) offset from it.  Interval ends include the
 * edge directions exactly, so theta - theta_e = (base - theta_e) + delta
 * keeps full relative accuracy even for rays within 1e-8 rad of an edge
 * direction (forming theta first would lose it). */
static double wrap_pi(double x) {
    if (x > OR_PI) x -= 2.0 * OR_PI;
    if (x < -OR_PI) x += 2.0 * OR_PI;
    return x;
}

static void ray(const octx *c, double base, double delta, double out[3]) {
    const otri *t = c->t;
    const double th = base + delta;
    double ct = cos(th), st = sin(th);
    double lo = 0.0, hi = INFINITY;
    for (int e = 0; e < 3; ++e) {
        /* inside: cross(b-a, x-a) >= 0 ; along x = r e_theta this reads
         * r |e| sin(theta - theta_e) >= cross(e, a); the sine is taken of the
         * angle to the nearer of the two edge directions */
        double d1 = wrap_pi(wrap_pi(base - t->eang[e]) + delta);
        double d2 = wrap_pi(wrap_pi(base - t->eopp[e]) + delta);
        double sn = fabs(d1) <= fabs(d2) ? sin(d1) : -sin(d2);
        double al = t->orient * t->elen[e] * sn;
        double be = t->orient * t->ecr[e];
        if (al > 0) { double r = be / al; if (r > lo) lo = r; }
        else if (al < 0) { double r = be / al; if (r < hi) hi = r; }
        else if (be > 0) { lo = 1.0; hi = 0.0; }
    }
    double v = 0.0, g = 0.0;
    for (int p = 0; p < c->K->npieces; ++p) {
        double r0 = lo, r1 = hi < c->K->R[p] ? hi : c->K->R[p];
        if (!(r1 > r0)) continue;
        double hw = 0.5 * (r1 - r0), md = 0.5 * (r1 + r0);
        for (int i = 0; i < c->nr; ++i) {
            double r = md + hw * gl_x[c->nr][i];
            double w = hw * gl_w[c->nr][i];
            double A = field_at(t, r * ct, r * st);
            v += w * A * kpiece(c->K, p, r) * r;
            g += w * A * kpiece_d(c->K, p, r) * r;
        }
    }
    out[0] = v;
    out[1] = -g * ct;
    out[2] = -g * st;
}

static void glq(const octx *c, double a, double b, int n, double q[3], double *qabs) {
    double hw = 0.5 * (b - a);
    q[0] = q[1] = q[2] = 0.0;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double o[3];
        double x = gl_x[n][i];
        if (x <= 0.0) ray(c, a, hw * (1.0 + x), o);      /* offsets from the nearer end */
        else ray(c, b, -hw * (1.0 - x), o);
        double w = hw * gl_w[n][i];
        q[0] += w * o[0]; q[1] += w * o[1]; q[2] += w * o[2];
        s += w * (fabs(o[0]) + fabs(o[1]) + fabs(o[2]));
    }
    if (qabs) *qabs = s;
}

/* Adaptive bisection.  An interval is accepted when the 10- and 20-point
 * rules agree to tol per unit angle, tol = 4e-15 times the field scale.  The
 * integrand itself carries absolute rounding noise of about 1e-15 per unit
 * angle (r_in and r_out come from ratios that are ill-conditioned for rays
 * nearly parallel to an edge), so a tighter tolerance would only refine
 * noise; the total error stays below 2.5e-14 times the field scale.  Depth
 * and call caps bound the work; an interval accepted at a cap marks the pair
 * as unverified (the entry points report it). */
static void adapt(octx *c, double a, double b, int depth, double acc[3]) {
    double q1[3], q2[3];
    glq(c, a, b, 10, q1, NULL);
    glq(c, a, b, 20, q2, NULL);
    double err = 0.0;
    for (int k = 0; k < 3; ++k) { double d = fabs(q2[k] - q1[k]); if (d > err) err = d; }
    const int converged = err <= c->tol * (b - a);
    if (converged || depth >= 40 || ++c->calls > 2000000) {
        if (!converged) c->capped = 1;
        acc[0] += q2[0]; acc[1] += q2[1]; acc[2] += q2[2];
        return;
    }
    double m = 0.5 * (a + b);
    adapt(c, a, m, depth + 1, acc);
    adapt(c, m, b, depth + 1, acc);
}

static int cmp_d(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* One pair in the normalised frame.  out = (int A k, -int A e k' ) without C_d.
 * Returns 1 when the adaptive rule stopped at a cap somewhere (the value is
 * then not verified to the stated tolerance), else 0. */
static int pair_normalised(const okern *K, otri *t, double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    double area2 = (t->x[1] - t->x[0]) * (t->y[2] - t->y[0]) - (t->x[2] - t->x[0]) * (t->y[1] - t->y[0]);
    if (area2 == 0.0 || !isfinite(area2)) return 0;         /* zero-area triangles contribute 0 */
    t->orient = area2 > 0 ? 1.0 : -1.0;                      /* inside test works for either orientation */
    for (int e = 0; e < 3; ++e) {
        int a = e, b = (e + 1) % 3;
        double ex = t->x[b] - t->x[a], ey = t->y[b] - t->y[a];
        t->elen[e] = sqrt(ex * ex + ey * ey);
        t->eang[e] = atan2(ey, ex);
        t->eopp[e] = atan2(-ey, -ex);
        t->ecr[e] = ex * t->y[a] - ey * t->x[a];
    }
    t->D = (t->y[1] - t->y[2]) * (t->x[0] - t->x[2]) + (t->x[2] - t->x[1]) * (t->y[0] - t->y[2]);
    double amax = 0.0;
    for (int i = 0; i < t->nn; ++i) amax = fmax(amax, fabs(t->A[i]));
    octx c = {K, t, 12, 0, 4e-15 * fmax(1.0, (t->nn == 10 ? 3.0 : 1.0) * amax), 0};
    double br[1024];
    int nb = 0;
    br[nb++] = -OR_PI;
    br[nb++] = OR_PI;
    for (int i = 0; i < 3; ++i) {
        if (t->x[i] != 0.0 || t->y[i] != 0.0) br[nb++] = atan2(t->y[i], t->x[i]);
        else {  /* vertex at the particle: the edge directions bound the span */
            for (int j = 0; j < 3; ++j)
                if (j != i) br[nb++] = atan2(t->y[j], t->x[j]);
        }
    }
    /* directions in which a ray is parallel to an edge line, or hits it at
     * the foot of the perpendicular: when the line passes close to the
     * particle the integrand turns sharply within ~p radians of these, so
     * they are made interval ends where the rules resolve the layer */
    for (int e = 0; e < 3; ++e) {
        br[nb++] = t->eang[e];
        br[nb++] = t->eopp[e];
        double fa = t->eang[e] + (t->ecr[e] > 0 ? -0.5 : 0.5) * OR_PI;
        br[nb++] = wrap_pi(fa);
        /* a line at distance p is met at r = p / sin(delta), delta the angle
         * to its direction: the integrand depends on log(delta) for
         * delta in [p, 1], so a geometric grading of breakpoints toward the
         * parallel directions lets the rules see that layer */
        double p = t->elen[e] > 0 ? fabs(t->ecr[e]) / t->elen[e] : 0.0;
        if (p > 0.0 && p < 0.05)
            for (double off = 0.25 * p; off < 0.2; off *= 2.0)
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    br[nb++] = wrap_pi(t->eang[e] + sgn * off);
                    br[nb++] = wrap_pi(t->eopp[e] + sgn * off);
                }
    }
    for (int p = 0; p < K->npieces; ++p) {
        double R = K->R[p];
        for (int e = 0; e < 3; ++e) {
            int a = e, b = (e + 1) % 3;
            double dx = t->x[b] - t->x[a], dy = t->y[b] - t->y[a];
            double A = dx * dx + dy * dy, B = 2.0 * (t->x[a] * dx + t->y[a] * dy);
            double C = t->x[a] * t->x[a] + t->y[a] * t->y[a] - R * R;
            double disc = B * B - 4 * A * C;
            if (disc <= 0 || A == 0) continue;
            double sq = sqrt(disc);
            double s[2] = {(-B - sq) / (2 * A), (-B + sq) / (2 * A)};
            for (int k = 0; k < 2; ++k)
                if (s[k] > 0.0 && s[k] < 1.0) {
                    double X = t->x[a] + s[k] * dx, Y = t->y[a] + s[k] * dy;
                    br[nb++] = atan2(Y, X);
                }
        }
    }
    qsort(br, nb, sizeof(double), cmp_d);
    for (int i = 0; i + 1 < nb; ++i) {
        if (br[i + 1] > br[i]) adapt(&c, br[i], br[i + 1], 0, out);
    }
    return c.capped;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* ------------------------------------------------------------------ */

/* One (particle, triangle) pair in world coordinates.
 * tri6 = x0,y0,x1,y1,x2,y2 ; A = nodal values (nn of them).
 * out = (I, Gx, Gy) including C_d and the 1/h of the gradient.
 * Returns 0, -1 for bad arguments, or 1 when the adaptive rule stopped at
 * its depth or call cap (out is written but unverified). */
int oracle_pair(int kernel_id, double h, int nn, double px, double py, const double *tri6,
                const double *A, double *out) {
    okern K;
    if (oracle_kernel(kernel_id, &K)) return -1;
    if (!(h > 0) || (nn != 1 && nn != 3 && nn != 10)) return -1;
    otri t;
    t.nn = nn;
    for (int i = 0; i < 3; ++i) {
        t.x[i] = (tri6[2 * i] - px) / h;       /* nu* = C nu (Sec. 2) */
        t.y[i] = (tri6[2 * i + 1] - py) / h;
    }
    for (int i = 0; i < nn; ++i) t.A[i] = A[i];
    double o[3];
    const int capped = pair_normalised(&K, &t, o);
    out[0] = K.Cd * o[0];
    out[1] = K.Cd * o[1] / h;
    out[2] = K.Cd * o[2] / h;
    return capped;
}

/* Same, with the triangle already in the support-normalised frame (h = 1). */
int oracle_pair_normalised(int kernel_id, int nn, const double *tri6, const double *A, double *out) {
    return oracle_pair(kernel_id, 1.0, nn, 0.0, 0.0, tri6, A, out);
}

/* Per-particle sums over a CSR pair list (eq. boundaryint).
 * tri: [6][T] SoA, nodal: [nn][T], per_pair (nullable): [3][P].
 * Returns 0; -1 for bad arguments; -2 if a triangle index is out of range;
 * otherwise the number of pairs whose adaptive rule stopped at a cap
 * (positive: all outputs are written, those pairs are unverified). */
int oracle_integrate(int kernel_id, double h, int nn, int64_t N, const double *px, const double *py,
                     int64_t T, const double *tri, const double *nodal, const int64_t *offsets,
                     const int32_t *tri_idx, double *I, double *Gx, double *Gy, double *per_pair,
                     int nthreads) {
    okern K;
    if (oracle_kernel(kernel_id, &K)) return -1;
    if (!(h > 0) || (nn != 1 && nn != 3 && nn != 10) || N < 0 || T < 0) return -1;
    int64_t P = N > 0 ? offsets[N] : 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int bad = 0;
    long capped = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(|:bad) reduction(+:capped)
    for (int64_t i = 0; i < N; ++i) {
        double si = 0, sx = 0, sy = 0;
        for (int64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
            int64_t j = tri_idx[q];
            if (j < 0 || j >= T) { bad = 1; continue; }
            otri t;
            t.nn = nn;
            for (int v = 0; v < 3; ++v) {
                t.x[v] = (tri[(2 * v) * T + j] - px[i]) / h;
                t.y[v] = (tri[(2 * v + 1) * T + j] - py[i]) / h;
            }
            for (int a = 0; a < nn; ++a) t.A[a] = nodal[a * T + j];
            double o[3];
            capped += pair_normalised(&K, &t, o);
            double vi = K.Cd * o[0], vx = K.Cd * o[1] / h, vy = K.Cd * o[2] / h;
            if (per_pair) { per_pair[q] = vi; per_pair[P + q] = vx; per_pair[2 * P + q] = vy; }
            si += vi; sx += vx; sy += vy;
        }
        I[i] = si; Gx[i] = sx; Gy[i] = sy;
    }
    if (bad) return -2;
    return capped > 0x7fffffff ? 0x7fffffff : (int)capped;
}

/* ------------------------------------------------------------------ */
/* pair enumeration by brute force: all (i, j) with dist(x_i, T_j) < h  */
/* ------------------------------------------------------------------ */
static double seg_d2(double px, double py, double ax, double ay, double bx, double by) {
    double dx = bx - ax, dy = by - ay;
    double L = dx * dx + dy * dy;
    double t = L > 0 ? ((px - ax) * dx + (py - ay) * dy) / L : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double ex = ax + t * dx - px, ey = ay + t * dy - py;
    return ex * ex + ey * ey;
}

double oracle_point_triangle_dist2(double px, double py, const double *t6) {
    double x0 = t6[0], y0 = t6[1], x1 = t6[2], y1 = t6[3], x2 = t6[4], y2 = t6[5];
    double c0 = (x1 - x0) * (py - y0) - (y1 - y0) * (px - x0);
    double c1 = (x2 - x1) * (py - y1) - (y2 - y1) * (px - x1);
    double c2 = (x0 - x2) * (py - y2) - (y0 - y2) * (px - x2);
    if ((c0 >= 0 && c1 >= 0 && c2 >= 0) || (c0 <= 0 && c1 <= 0 && c2 <= 0)) return 0.0;
    double d = seg_d2(px, py, x0, y0, x1, y1);
    double e = seg_d2(px, py, x1, y1, x2, y2);
    double f = seg_d2(px, py, x2, y2, x0, y0);
    if (e < d) d = e;
    if (f < d) d = f;
    return d;
}

/* Pass 1 (tri_idx == NULL): counts into offsets[i+1]; pass 2 fills tri_idx
 * in ascending triangle order.  Returns the number of pairs. */
int64_t oracle_pairlist(int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                        double h, int64_t *offsets, int32_t *tri_idx, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double h2 = h * h;
    if (!tri_idx) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < N; ++i) {
            int64_t c = 0;
            for (int64_t j = 0; j < T; ++j) {
                double t6[6];
                for (int k = 0; k < 6; ++k) t6[k] = tri[k * T + j];
                if (oracle_point_triangle_dist2(px[i], py[i], t6) < h2) ++c;
            }
            offsets[i + 1] = c;
        }
        offsets[0] = 0;
        for (int64_t i = 0; i < N; ++i) offsets[i + 1] += offsets[i];
        return offsets[N];
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        int64_t q = offsets[i];
        for (int64_t j = 0; j < T; ++j) {
            double t6[6];
            for (int k = 0; k < 6; ++k) t6[k] = tri[k * T + j];
            if (oracle_point_triangle_dist2(px[i], py[i], t6) < h2) tri_idx[q++] = (int32_t)j;
        }
    }
    return offsets[N];
}
