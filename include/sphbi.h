/*
 * sphbi.h -- analytic SPH boundary integrals on AMD Instinct MI355X (gfx950).
 *
 * For every (particle, boundary triangle) pair inside the kernel support the
 * library evaluates, in closed form,
 *
 *     I(x) = int_T A_T(x') W(|x - x'|) dx'          (Sec. 2, eq. sphintegral,
 *     G(x) = int_T A_T(x') grad_x W(|x - x'|) dx'    eq. nablaIntegral, eq. boundaryint)
 *
 * for a compact polynomial kernel W(r) = c_d h^-2 k(r/h) (Sec. 2) and a
 * polynomial field A_T on the triangle (Sec. 3): constant (1 value per
 * triangle), linear (3 vertex values, barycentric interpolation) or cubic
 * Lagrange (10 values).  Per particle the results are summed over its
 * triangles (eq. boundaryint).  Each pair is decomposed into
 * particle-anchored pieces (Sec. 4) evaluated with Chebyshev angular terms and
 * the hypergeometric radial term (Sec. 5).
 *
 * Conventions
 *  - h is the support radius: W vanishes for |x - x'| >= h.
 *  - All array arguments are DEVICE pointers owned by the caller unless the
 *    argument says "host".  Nothing is freed by the library.  Calls are
 *    asynchronous on `stream` (a hipStream_t; NULL = default stream) unless
 *    documented as synchronising.
 *  - Arrays are structure-of-arrays, float64, 8-byte aligned:
 *      px, py            [N]
 *      tri               [6][T]  rows x0, y0, x1, y1, x2, y2
 *      nodal             [n_nodes][T]
 *      offsets           int64 [N+1] CSR row pointer (pairs of particle i are
 *                        offsets[i] .. offsets[i+1]-1)
 *      tri_idx           int32 [P]   triangle of each pair
 *      I, Gx, Gy         [N]
 *      per_pair          [3][P] rows I, Gx, Gy (optional, may be NULL)
 *  - Cubic node order: v0, v1, v2; edge v0->v1 at 1/3 and 2/3; edge v1->v2 at
 *    1/3, 2/3; edge v2->v0 at 1/3, 2/3; centroid.
 *  - Zero-area triangles contribute 0.  Either vertex orientation gives the
 *    same result.  Overlapping triangles are summed, not checked (Sec. 2).
 *  - Pairs of tri_idx outside [offsets[0], offsets[N]) belong to no particle:
 *    they contribute nothing to any output (their per_pair slots are left
 *    as they were).  Offsets must be non-decreasing; offsets outside [0, P]
 *    are clamped, so a malformed list never makes a kernel read out of
 *    bounds.
 *  - One call handles at most 2^28 - 256 particles and as many triangles
 *    (every launch's grid must fit a 32-bit thread count); larger sizes
 *    return SPHBI_EUNSUPPORTED before any launch.
 *  - Return value: SPHBI_OK or a negative status; sphbi_last_error() gives a
 *    message (thread-local).
 */
#ifndef SPHBI_H
#define SPHBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPHBI_OK 0
#define SPHBI_EINVAL -1       /* bad argument (null pointer, h <= 0, sizes, degree, n_nodes) */
#define SPHBI_EUNSUPPORTED -2 /* valid but not implemented combination */
#define SPHBI_EDEVICE -3      /* HIP launch or runtime error */
#define SPHBI_ENOWORKSPACE -4 /* workspace missing or too small */
#define SPHBI_ECAPACITY -5    /* output capacity too small (count returned) */
#define SPHBI_EGRID -6        /* a particle lies outside the grid being reused: plan again */

#define SPHBI_WENDLAND_C2 0
#define SPHBI_WENDLAND_C4 1
#define SPHBI_WENDLAND_C6 2
#define SPHBI_CUBIC_BSPLINE 3

#define SPHBI_FP64 0
#define SPHBI_MIXED 1

#define SPHBI_REFINE_AUTO 0 /* double-double for the pairs the conditioning gate selects (default) */
#define SPHBI_REFINE_OFF 1  /* every pair in the precision mode alone */
#define SPHBI_REFINE_ALL 2  /* every pair in double-double (slow; a reference on the device) */

/* Kernel k(q) = sum_p [q < radius[p]] sum_k b[p][k] q^k (q = r/h), with
 * W(r) = c_d h^-2 k(r/h) (Sec. 2: compact polynomial kernels; piecewise
 * kernels such as B-splines are handled piece by piece).  n_pieces 1 or 2,
 * degree[p] <= 11, 0 < radius[p] <= 1. */
typedef struct {
    int32_t n_pieces;
    int32_t degree[2];
    int32_t reserved;
    double radius[2];
    double b[2][12];
    double c_d;
} sphbi_kernel;

/* Refinement of ill-conditioned pairs (sphbi_integrate and
 * sphbi_integrate_noalloc).  For a linear or cubic field the particle-anchored
 * pieces of the decomposition (Sec. 4) extend the field polynomial from the
 * triangle to the particle, and its harmonics about the particle (Sec. 3)
 * exceed the integrand by the factor kappa^order, kappa = d_max l_max /
 * |2 area| (d_max the farthest vertex from the particle, l_max the longest
 * edge); FP64 then loses about Kf kappa^order in relative accuracy, Kf =
 * sum|b_k|/(k+2) / |sum b_k/(k+2)| the cancellation of the kernel's monomial
 * form (141 for Wendland C2, 1109 C4, 8704 C6, 30 B-spline).  With
 * SPHBI_REFINE_AUTO the pairs with Kf kappa^order > refine_gate are left out of
 * the FP64 (or mixed) pass and evaluated in double-double from the input
 * doubles, then added in pair order; results stay deterministic.  Constant
 * fields are never refined. */
typedef struct {
    int32_t precision;  /* SPHBI_FP64 or SPHBI_MIXED */
    int32_t refine;     /* SPHBI_REFINE_AUTO (default), _OFF or _ALL */
    double tau_edge;    /* MIXED: pairs whose particle lies within tau_edge*h of an
                           edge line or vertex are evaluated in FP64 (default 1e-4) */
    double refine_gate; /* threshold on Kf kappa^order; 0 = the default,
                           FP64: G0 (141/Kf)^1.65 with G0 = 3e6 for cubic and 3e8
                           for linear fields; MIXED: 1e9 (141/Kf)^1.25 */
    uint8_t *pair_status; /* optional DEVICE array [n_pairs] (sphbi_integrate, _noalloc,
                             _prepared): per pair 1 if any of its three results is not
                             finite (NaN or Inf from degenerate or non-finite input), else 0;
                             pairs outside [offsets[0], offsets[N]) are left as they were.
                             NULL (the default) writes nothing. */
} sphbi_opts;

/* Fills *out with a preset kernel: Wendland C2 (1-q)^4(1+4q), C4
 * (1-q)^6(1+6q+35/3 q^2), C6 (1-q)^8(1+8q+25q^2+32q^3), cubic B-spline
 * (1-q)^3 - 4(1/2-q)^3_+; c_d normalises the kernel to unit integral over the
 * support disc.  Host only. */
int sphbi_kernel_preset(int32_t id, sphbi_kernel *out);

/* Default options (FP64, tau_edge = 1e-4).  Host only. */
void sphbi_default_opts(sphbi_opts *out);

/* Message of the last failing call on this thread. */
const char *sphbi_last_error(void);

/* ---------------------------------------------------------------------
 * Pair enumeration (the neighbour set N_T of Sec. 2, eq. boundaryint):
 * pairs (i, j) with dist(x_i, T_j) < h, grouped by particle, triangles in
 * ascending index order within a particle.
 *
 * sphbi_pairlist_plan: sizes the uniform cell grid (cell >= h) over the
 * particles' bounding box and returns the workspace the two later calls need.
 * A particle coordinate that is not finite returns SPHBI_EINVAL.
 * Synchronises `stream`.
 *
 * sphbi_pairlist_count: builds the grid in `ws`, counts the pairs of every
 * particle and writes offsets[0..N]; *n_pairs (host) receives offsets[N].
 * Synchronises `stream`.
 *
 * sphbi_pairlist_recount: sphbi_pairlist_count for new particle positions on
 * a grid and cell lists built before, for a mesh that has not moved (same
 * tri, T and h as the count call that built `ws`, which must not have been
 * overwritten since).  N may differ from that call's; ws_bytes must then
 * still cover the layout sphbi_pairlist_plan would give for the new N on
 * this grid (it does whenever N did not grow).  Skips the cell lists' build
 * (about a third of the three calls' time on a million particles).  If any
 * particle lies outside the grid's nx x ny cells, or has a non-finite
 * coordinate, the offsets written are incomplete and the call returns
 * SPHBI_EGRID: plan and count again.  The result is identical to a fresh
 * plan + count on the same grid.  Synchronises `stream`.
 *
 * sphbi_pairlist_fill: writes tri_idx[0 .. n_pairs-1] using the offsets and
 * the grid, cell lists and per-particle candidate masks left in `ws` by the
 * count call.  cap is the length of tri_idx; cap < offsets[N] returns
 * SPHBI_ECAPACITY, for which it reads offsets[N] back and so synchronises
 * `stream`.
 * ------------------------------------------------------------------- */
typedef struct {
    double x0, y0, cell;
    int32_t nx, ny;
    int64_t n_refs; /* triangle-to-cell registrations */
} sphbi_grid;

int sphbi_pairlist_plan(int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                        double h, sphbi_grid *grid /* host out */, size_t *ws_bytes /* host out */,
                        void *stream);
int sphbi_pairlist_count(int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                         double h, const sphbi_grid *grid /* host */, void *ws, size_t ws_bytes,
                         int64_t *offsets, int64_t *n_pairs /* host out */, void *stream);
int sphbi_pairlist_recount(int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                           double h, const sphbi_grid *grid /* host */, void *ws, size_t ws_bytes,
                           int64_t *offsets, int64_t *n_pairs /* host out */, void *stream);
int sphbi_pairlist_fill(int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                        double h, const sphbi_grid *grid /* host */, void *ws, size_t ws_bytes,
                        const int64_t *offsets, int32_t *tri_idx, int64_t cap, void *stream);

/* ---------------------------------------------------------------------
 * Forward integrals (eq. boundaryint and its gradient; Sec. 3-5).
 *
 * sphbi_integrate_workspace: bytes of device workspace sphbi_integrate needs
 * for T triangles: per-triangle field records (128 B each), the refinement
 * pass's counters (256 B: pairs left out, windows handed out), and its
 * double-double records (256 B each).  Host only.
 *
 * sphbi_integrate: I, Gx, Gy [N] per particle = sum over its pairs; if
 * per_pair is not NULL also the per-pair values [3][P].  Positions and h in
 * world units; the gradient carries the 1/h of the normalisation (Sec. 2).
 * ws/ws_bytes: device workspace of at least sphbi_integrate_workspace(T)
 * bytes; the call overwrites it.  Asynchronous.
 * ------------------------------------------------------------------- */
size_t sphbi_integrate_workspace(int64_t T);

int sphbi_integrate(const sphbi_kernel *kernel /* host */, const sphbi_opts *opts /* host, NULL = default */,
                    double h, int32_t n_nodes, int64_t N, const double *px, const double *py, int64_t T,
                    const double *tri, const double *nodal, const int64_t *offsets, const int32_t *tri_idx,
                    int64_t n_pairs, double *I, double *Gx, double *Gy, double *per_pair, void *ws,
                    size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * sphbi_integrate without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation).  Same arguments, results and status codes as
 * sphbi_integrate, minus ws/ws_bytes.  The per-triangle field records go to
 * a fixed array inside this library (one copy per GPU, allocated with the
 * code object and held until the process ends) of SPHBI_NOALLOC_MAX_TRIANGLES
 * records, 48 MiB with the refinement pass's counters and double-double
 * records; T above that returns SPHBI_EUNSUPPORTED and launches
 * nothing.  No call allocates or frees memory.  The first call on a device
 * looks up that device's array address (synchronous, once per device).
 * Every call on one GPU shares its array: calls that overlap in time on
 * the same GPU (different streams or threads) race and must be ordered by
 * the caller.  Asynchronous.
 * ------------------------------------------------------------------- */
#define SPHBI_NOALLOC_MAX_TRIANGLES 131072

int sphbi_integrate_noalloc(const sphbi_kernel *kernel /* host */, const sphbi_opts *opts /* host, NULL = default */,
                            double h, int32_t n_nodes, int64_t N, const double *px, const double *py, int64_t T,
                            const double *tri, const double *nodal, const int64_t *offsets, const int32_t *tri_idx,
                            int64_t n_pairs, double *I, double *Gx, double *Gy, double *per_pair, void *stream);

/* ---------------------------------------------------------------------
 * The two stages of sphbi_integrate, for callers that reuse the per-triangle
 * field records across calls (static boundary, repeated evaluation) or time
 * the pair kernel alone.
 *
 * sphbi_field_prepare: writes T records of 16 doubles into rec (device,
 * at least sphbi_integrate_workspace(T) bytes): the vertices and the field
 * of every triangle as a polynomial about its first vertex (Sec. 3:
 * barycentric / FEM-stencil fields are polynomials).  Asynchronous.
 *
 * sphbi_integrate_prepared: the pair kernel of sphbi_integrate on records
 * written by sphbi_field_prepare with the same h and n_nodes.  Asynchronous.
 * ------------------------------------------------------------------- */
int sphbi_field_prepare(double h, int32_t n_nodes, int64_t T, const double *tri, const double *nodal, double *rec,
                        size_t rec_bytes, void *stream);
int sphbi_integrate_prepared(const sphbi_kernel *kernel /* host */, const sphbi_opts *opts /* host, NULL = default */,
                             double h, int32_t n_nodes, int64_t N, const double *px, const double *py, int64_t T,
                             const double *rec, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs,
                             double *I, double *Gx, double *Gy, double *per_pair, void *stream);

/* ---------------------------------------------------------------------
 * Numerical quadrature of the same sums as sphbi_integrate (the comparison
 * of the closed form with quadrature rules, Sec. 6.1-6.2).
 *
 * Every pair's triangle is integrated with a collapsed (Duffy) tensor
 * Gauss-Legendre rule of n_gauss x n_gauss points: barycentric L1 = u,
 * L2 = (1 - u) v, area element |2 area| (1 - u) du dv; exact for the field
 * times polynomials of total degree <= 2 n_gauss - 2, but the kernel's
 * compact cut-off and its odd powers of |x - x'| are not polynomials, which
 * limits the accuracy (Sec. 6.1).  Arguments, layouts and outputs as
 * sphbi_integrate (I, Gx, Gy [N], world units, the gradient with its 1/h);
 * 1 <= n_gauss <= SPHBI_MAX_GAUSS, else SPHBI_EINVAL.  FP64, no workspace,
 * deterministic (pairs summed in order).  Asynchronous.
 * ------------------------------------------------------------------- */
#define SPHBI_MAX_GAUSS 64

int sphbi_integrate_quadrature(const sphbi_kernel *kernel /* host */, double h, int32_t n_nodes, int32_t n_gauss,
                               int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                               const double *nodal, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs,
                               double *I, double *Gx, double *Gy, void *stream);

/* ---------------------------------------------------------------------
 * Adjoint (vector-Jacobian product) of sphbi_integrate.
 *
 * Given cotangents gI, gGx, gGy [N] of the per-particle outputs, writes the
 * gradients of L = sum_i gI_i I_i + gGx_i Gx_i + gGy_i Gy_i with respect to
 *   dpx, dpy  [N]           particle positions,
 *   dtri      [6][T]        triangle vertex coordinates (same layout as tri),
 *   dnodal    [n_nodes][T]  nodal field values.
 * The clipping and decomposition are recomputed, nothing is stored by the
 * forward call.  Deterministic: triangle sums are taken in pair order.
 * ws: device workspace of sphbi_integrate_backward_workspace(T, n_pairs,
 * n_nodes) bytes.  FP64 only.  Asynchronous.
 * ------------------------------------------------------------------- */
size_t sphbi_integrate_backward_workspace(int64_t T, int64_t n_pairs, int32_t n_nodes);

int sphbi_integrate_backward(const sphbi_kernel *kernel /* host */, const sphbi_opts *opts /* host, NULL = default */,
                             double h, int32_t n_nodes, int64_t N, const double *px, const double *py, int64_t T,
                             const double *tri, const double *nodal, const int64_t *offsets, const int32_t *tri_idx,
                             int64_t n_pairs, const double *gI, const double *gGx, const double *gGy, double *dpx,
                             double *dpy, double *dtri, double *dnodal, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * SPH operators on the boundary (Sec. 2) and the boundary normal (App. A).
 *
 * One call evaluates, for every particle x, op applied to boundary fields
 * given by nodal values on the triangles ([n_nodes][T], the layout of
 * sphbi_integrate), summed over the particle's pairs:
 *
 *   SPHBI_OP_GRAD_DIFFERENCE  (out_a, out_b) = difference gradient of A
 *       (eq. sphdiffops, first form; continuous form eq. intsphdiffops):
 *       (1/rho(x)) int f grad W, f interpolated from the pre-weights
 *       f_i = rho_i (A_i - A(x)) at the element's nodes.
 *       fa = A, fb = rho (nodal); qa = A(x), qb = rho(x) [N].
 *   SPHBI_OP_GRAD_SYMMETRIC   (out_a, out_b) = symmetric gradient of A:
 *       rho(x) int f grad W, f_i = rho_i (A_i / rho_i^2 + A(x) / rho(x)^2)
 *       (the sign of the pre-weights given with eq. improper and used in
 *       App. A for the pressure term).  Same arguments.
 *   SPHBI_OP_DIV_CURL         out_a = divergence, out_b = curl of the vector
 *       field (A_x, A_y): <grad A_x>_x + <grad A_y>_y and
 *       <grad A_y>_x - <grad A_x>_y.  fa = A_x, fb = A_y; qa, qb unused.
 *   SPHBI_OP_NORMAL           (out_a, out_b) = int grad W (the unit field;
 *       App. A).  n_nodes, fa, fb, qa, qb unused.
 *
 * "grad" is with respect to the particle position (as G of
 * sphbi_integrate, 1/h included).  Densities must be non-zero.  Pair list,
 * kernel and h as in sphbi_integrate.  ws: device workspace of
 * sphbi_operator_workspace(N, T) bytes (two per-triangle records and two
 * per-particle arrays); the call overwrites it.  FP64 only (opts may be
 * NULL; MIXED is rejected with SPHBI_EUNSUPPORTED).  Asynchronous.
 * ------------------------------------------------------------------- */
#define SPHBI_OP_GRAD_DIFFERENCE 0
#define SPHBI_OP_GRAD_SYMMETRIC 1
#define SPHBI_OP_DIV_CURL 2
#define SPHBI_OP_NORMAL 3

size_t sphbi_operator_workspace(int64_t N, int64_t T);

int sphbi_operator(const sphbi_kernel *kernel /* host */, const sphbi_opts *opts /* host, NULL = default */,
                   int32_t op, double h, int32_t n_nodes, int64_t N, const double *px, const double *py,
                   const double *qa, const double *qb, int64_t T, const double *tri, const double *fa,
                   const double *fb, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, double *out_a,
                   double *out_b, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Boundary pressure acceleration with one pressure value per contact
 * (App. A, the second choice for the boundary pressure): for every particle
 *   a_i = - sum over its pairs q of rho0 (p_q / rho0^2 + p_i / rho_i^2) int_T grad W,
 * with rho0 the (constant) rest density of the boundary, p_q the pressure at
 * the particle's closest point on the pair's triangle, one value per pair in
 * the order of tri_idx (the caller evaluates it, e.g. by MLS), and p_i, rho_i
 * the particle's pressure and density [N].  Output (ax, ay) [N].  The
 * per-vertex variant of App. A is minus the symmetric gradient of
 * sphbi_operator with rho = rho0 at the nodes, divided by rho_i.
 * ws: sphbi_operator_workspace(N, T) bytes.  FP64 only.  Asynchronous.
 * ------------------------------------------------------------------- */
int sphbi_pressure_contact(const sphbi_kernel *kernel /* host */, const sphbi_opts *opts /* host, NULL = default */,
                           double h, double rho0, int64_t N, const double *px, const double *py,
                           const double *p_particle, const double *rho_particle, int64_t T, const double *tri,
                           const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, const double *p_pair,
                           double *ax, double *ay, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Learned surrogate of the per-pair result (an extension; the paper has no
 * learned part).  A network 8 -> 128 -> 128 -> 128 -> 4 maps the
 * canonical features of a pair to the standardised (I, h Gx, h Gy) of a unit
 * P0 field in a rotated support-normalised frame (Sec. 2, transform C) plus
 * an error indicator (log10 of its own expected scaled error); between
 * layers the activation z s(u), s(u) = 1/2 + u/4 - u|u|/32, u = clamp(z, -4,
 * 4), a piecewise quadratic stand-in for z sigmoid(z).  Products run
 * on the matrix cores in bfloat16 with FP32 accumulation; master weights,
 * gradients and Adam moments are FP32.
 *
 * Parameters: one FP32 vector of SPHBI_MLP_PARAMS values, W1[8][128] b1[128]
 * W2[128][128] b2[128] W3[128][128] b3[128] W4[128][4] b4[4], W[in][out].
 * ------------------------------------------------------------------- */
#define SPHBI_MLP_PARAMS 34692

/* Canonical features of every pair of a CSR pair list: feats [n_pairs][8]
 * (rotated vertex coordinates in units of h, then (#vertices with |nu| <= 1)/3
 * and (#edges meeting the circle |nu| = 1)/3) and rot [n_pairs][2] = (cos,
 * sin) of the frame rotation; the first vertex of the canonical order (the
 * nearest to the particle) lies on the rotated +x axis.  Invalid triangle
 * indices give zero features.  Asynchronous. */
int sphbi_surrogate_features(double h, int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                             const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, float *feats,
                             float *rot, void *stream);

/* Training targets from closed-form per-pair values per_pair [3][n_pairs]
 * (sphbi_integrate with a unit P0 field): targets [n_pairs][3] =
 * ((I, h Gx', h Gy') - mean) / stdev, with (Gx', Gy') the gradient in the
 * frame rotated by rot (as written by sphbi_surrogate_features).  mean and
 * stdev are host arrays of 3.  Asynchronous. */
int sphbi_surrogate_targets(int64_t n_pairs, double h, const double *per_pair, const float *rot,
                            const float *mean /* host [3] */, const float *stdev /* host [3] */, float *targets,
                            void *stream);

/* Device workspace of the training calls for a batch of B rows.  Host only. */
size_t sphbi_mlp_workspace(int64_t B);

/* Network outputs out [B][4] for features feats [B][8] (all device).  Asynchronous. */
int sphbi_mlp_forward(const float *params, int64_t B, const float *feats, float *out, void *ws, size_t ws_bytes,
                      void *stream);

/* Loss and gradient of a batch:
 *   L = sum_b sum_{k<3} (y_bk - t_bk)^2 / (3B) + lam sum_b (y_b3 - e_b)^2 / B,
 *   e_b = log10(max_k |y_bk - t_bk| scale_k + 1e-7)   (held constant),
 * with y the network outputs, t = targets [B][3] (standardised) and scale
 * [3] (host) converting standardised units into the scale-normalised error.
 * Writes *loss (device, one float) and grad [SPHBI_MLP_PARAMS] (device,
 * overwritten).  Deterministic.  Asynchronous. */
int sphbi_mlp_loss_grad(const float *params, int64_t B, const float *feats, const float *targets,
                        const float *scale /* host [3] */, float lam, float *loss, float *grad, void *ws,
                        size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba, Algorithm 1, bias-corrected; `step` counts
 * from 1) on n FP32 parameters with moments m, v (device, updated in place). */
int sphbi_adam_step(float *params, float *m, float *v, const float *grad, int64_t n, double lr, double beta1,
                    double beta2, double eps, int64_t step, void *stream);

/* Serving model: the parameters rearranged for the fused kernel plus the
 * output standardisation (mean, stdev of the three targets) and the trained
 * feature range fmax.  sphbi_surrogate_model_bytes() bytes of device memory;
 * sphbi_surrogate_pack fills it.  Asynchronous. */
size_t sphbi_surrogate_model_bytes(void);
int sphbi_surrogate_pack(const float *params, const float *mean /* host [3] */, const float *stdev /* host [3] */,
                         float fmax, void *model, void *stream);

/* Device workspace of sphbi_surrogate_integrate.  Host only. */
size_t sphbi_surrogate_workspace(int64_t T, int64_t n_pairs);

/* Per-particle integrals of a P0 field (nodal [T], one value per triangle)
 * with the surrogate: a pair whose indicator exceeds `threshold`, or whose
 * features leave the trained range, is flagged and evaluated in closed form
 * (FP64) with `kernel` instead.  I, Gx, Gy [N] as sphbi_integrate; per_pair
 * [3][n_pairs] optional; flags [n_pairs] (1 = evaluated in closed form);
 * *n_flagged (device int64) receives their number.  The network is only
 * meaningful for the kernel it was trained with.  Deterministic.
 * Asynchronous. */
int sphbi_surrogate_integrate(const sphbi_kernel *kernel /* host */, double h, int64_t N, const double *px,
                              const double *py, int64_t T, const double *tri, const double *nodal,
                              const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, const void *model,
                              float threshold, double *I, double *Gx, double *Gy, double *per_pair, uint8_t *flags,
                              int64_t *n_flagged, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Measurement probe (not part of the method): the device's FP64 vector FMA
 * rate, against which the pair kernels' FP64 rates are compared.  Launches
 * eight waves per SIMD, each lane running 8 independent chains of `iters`
 * dependent fused multiply-adds (1 <= iters <= 2^24, else SPHBI_EINVAL).
 * *flops (host) receives the FP64 operations the launch executes (an FMA
 * counts two); time the launch on `stream` to get the rate.  sink: one
 * device double, never written in practice (it keeps the chains live).
 * Asynchronous.
 * ------------------------------------------------------------------- */
int sphbi_probe_fp64_fma(int64_t iters, double *sink, double *flops /* host out */, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPHBI_H */
