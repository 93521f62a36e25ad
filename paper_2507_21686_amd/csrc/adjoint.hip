// Adjoint of the forward integrals: given cotangents (gI, gGx, gGy) per
// particle, gradients with respect to particle positions, triangle vertices
// and nodal field values.
//
// With the cotangent-weighted kernel Phi(x) = gI W + gGx dW/dx_p + gGy dW/dy_p
// a pair contributes L = int_T A Phi dx.  Nothing from the forward pass is
// stored; every pair recomputes its field and clipping.
//   * Vertices (Reynolds transport, the Leibniz rule for a moving domain):
//     moving vertex k by e_alpha moves the boundary with velocity
//     lambda_k e_alpha (lambda_k its barycentric hat) and, the nodes moving
//     with the triangle, changes the field at a fixed point by
//     -lambda_k dA/dx_alpha, so
//       dL/dv_k,alpha = oint_dT A Phi lambda_k n_alpha ds
//                       + int_T (-lambda_k dA/dx_alpha) Phi dx.
//     Along an edge the boundary integral is a polynomial in the edge
//     coordinate times the kernel and its derivative, which reduce to the
//     radial terms H_c = int rho^(c-1) dy and powers of rho used by the forward
//     pass (edge_line below).
//   * Nodal values and the field part of the vertex term are linear in the
//     field: both follow from the moments m_j = int_T xi^j Phi dx of the
//     monomials about the particle.  The closed form is linear in the field's
//     harmonics, so pair_dual gets all of them in one pass; the nodal
//     gradients are the moments carried back through the shift to the
//     particle and the field preparation (their transposes).
//   * The particle gradient follows from translation invariance:
//     d/dx = -(d/dv0 + d/dv1 + d/dv2).
//
// Particle gradients are summed per particle with the forward kernel's
// segmented wave scan.  Per-pair triangle gradients go to a buffer and are
// summed per triangle in pair order through a stable sort by triangle index,
// so the whole adjoint is deterministic.

#include <math.h>

#include <hipcub/hipcub.hpp>

#include "internal.h"
#include "pairmath.h"

namespace sphbi {
namespace {

// Boundary term of one edge: with the particle at the origin (units of h), the
// edge on the line p n + y tau (tau = (-ny, nx)) from y = ya (vertex a) to
// y = yb (vertex b) and the field A given about the particle by c,
//   Ja = int (1 - t) A Phi ds,   Jb = int t A Phi ds   (t = (y - ya)/(yb - ya)),
// over the parts of the edge inside each kernel piece, in world units.
template <int DEG, int ORDER>
__device__ inline void edge_line(const KArgs &K, double p, double ya, double yb, double nx, double ny,
                                 const double *__restrict__ c, double gI, double gX, double gY, double invh,
                                 double &Ja, double &Jb) {
    constexpr int NP = ORDER + 2;                 // t A has degree ORDER + 1
    constexpr int NQ = ORDER + 3;                 // t A (p gn + y gt) has degree ORDER + 2
    Ja = Jb = 0.0;
    // A along the line: xi_x = p nx - y ny, xi_y = p ny + y nx
    double X[4][4], Y[4][4];                      // coefficients of X^i, Y^j in y
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) X[i][q] = Y[i][q] = 0.0;
    X[0][0] = Y[0][0] = 1.0;
#pragma unroll
    for (int i = 1; i <= ORDER; ++i)
#pragma unroll
        for (int q = 0; q <= i; ++q) {
            X[i][q] = p * nx * X[i - 1][q] + (q > 0 ? -ny * X[i - 1][q - 1] : 0.0);
            Y[i][q] = p * ny * Y[i - 1][q] + (q > 0 ? nx * Y[i - 1][q - 1] : 0.0);
        }
    double Ay[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m <= ORDER; ++m)
#pragma unroll
        for (int j = 0; j <= m; ++j) {
            const int i = m - j;
            const double cij = c[pidx(i, j)];
#pragma unroll
            for (int qa = 0; qa <= i; ++qa)
#pragma unroll
                for (int qb = 0; qb <= j; ++qb) Ay[qa + qb] += cij * X[i][qa] * Y[j][qb];
        }
    // Pb = t A, Pa = A - Pb
    const double il = 1.0 / (yb - ya);
    double Pa[NP], Pb[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const double prev = q > 0 ? Ay[q - 1] : 0.0;
        const double cur = q <= ORDER ? Ay[q] : 0.0;
        Pb[q] = il * (prev - ya * cur);
        Pa[q] = cur - Pb[q];
    }
    // gX xi_x + gY xi_y = p gn + y gt
    const double gn = gX * nx + gY * ny, gt = -gX * ny + gY * nx;
    double Qa[NQ], Qb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        Qa[q] = (q < NP ? p * gn * Pa[q] : 0.0) + (q > 0 ? gt * Pa[q - 1] : 0.0);
        Qb[q] = (q < NP ? p * gn * Pb[q] : 0.0) + (q > 0 ? gt * Pb[q - 1] : 0.0);
    }
    const double lo0 = fmin(ya, yb), hi0 = fmax(ya, yb);
    const double p2 = p * p;
    // y^a = y^(a mod 2) (rho^2 - p^2)^m, m = a div 2, so every term reduces to
    // int rho^c dy = H_(c+1) (H_c = int rho^(c-1) dy, the forward pass's radial
    // terms) and int y rho^c dy = E_(c+2), E_e = (rho_hi^e - rho_lo^e)/e.  With
    // the kernel folded in first,
    //   int y^a W dy          = sum_i C(m,i) (-p^2)^(m-i) (a even ? G0[i] : G1[i]),
    //   int y^a W'/rho dy * h = sum_i C(m,i) (-p^2)^(m-i) (a even ? K0[i] : K1[i]),
    //   G0[i] = sum_j b_j H_(2i+j+1),  G1[i] = sum_j b_j E_(2i+j+2),
    //   K0[i] = sum_j j b_j H_(2i+j-1), K1[i] = sum_j j b_j E_(2i+j),
    // and the sums over j are taken while H and E are generated, so neither is
    // stored.
    constexpr int MI = (NQ - 1) / 2;              // largest m
    constexpr int HL = DEG + 2 * MI + 2;          // largest radial index used
#pragma unroll
    for (int pc = 0; pc < 2; ++pc) {
        if (pc >= K.npieces) break;
        const double R = K.R[pc];
        if (!(p < R)) continue;
        const ExactMath math;
        const double yc = math.sqrt_((R - p) * (R + p));
        const double lo = fmax(lo0, -yc), hi = fmin(hi0, yc);
        if (!(lo < hi)) continue;
        const double rl = math.sqrt_(p2 + lo * lo), rh = math.sqrt_(p2 + hi * hi);
        double G0[MI + 1], G1[MI + 1], K0[MI + 1], K1[MI + 1];
#pragma unroll
        for (int i = 0; i <= MI; ++i) G0[i] = G1[i] = K0[i] = K1[i] = 0.0;
        // H_0 = asinh(hi/p) - asinh(lo/p), only ever multiplied by p or p^2,
        // so 0 on a line through the particle
        const double H0 = p > 0.0 ? math.h0(p, lo, hi, rl, rh) : 0.0;
        double hm2 = 0.0, hm1 = 0.0;              // H_(c-2), H_(c-1)
        double gl = 1.0, gh = 1.0;                // rho^(c-1)
        double el = 1.0, eh = 1.0;                // rho^e
#pragma unroll
        for (int c = 0; c <= HL; ++c) {
            double Hc;
            if (c == 0) {
                Hc = H0;
            } else if (c == 1) {
                Hc = hi - lo;
            } else {
                gl *= rl;
                gh *= rh;
                Hc = (gh * hi - gl * lo + lit(c - 1.0) * p2 * hm2) * lit(1.0 / c);
            }
            double Ec = 0.0;
            if (c >= 1) {
                el *= rl;
                eh *= rh;
                Ec = (eh - el) * lit(1.0 / c);
            }
#pragma unroll
            for (int i = 0; i <= MI; ++i) {
                const int j0 = c - 2 * i - 1, j1 = c - 2 * i - 2, k0 = c - 2 * i + 1, k1 = c - 2 * i;
                if (j0 >= 0 && j0 <= DEG) G0[i] = fma(K.b[pc][j0], Hc, G0[i]);
                if (j1 >= 0 && j1 <= DEG && c >= 1) G1[i] = fma(K.b[pc][j1], Ec, G1[i]);
                if (k0 >= 1 && k0 <= DEG) K0[i] = fma(lit(k0) * K.b[pc][k0], Hc, K0[i]);
                if (k1 >= 1 && k1 <= DEG && c >= 1) K1[i] = fma(lit(k1) * K.b[pc][k1], Ec, K1[i]);
            }
            hm2 = hm1;
            hm1 = Hc;
        }
        // int y^a (W or W') dy for every power a of the field polynomials
        auto expand = [&](int a, const double *g0, const double *g1) -> double {
            const int m = a >> 1;
            const double *g = (a & 1) ? g1 : g0;
            double s = 0.0, pw = 1.0;
#pragma unroll
            for (int i = 2; i >= 0; --i) {
                if (i > m) continue;
                const double w = (m == 2 && i == 1 ? 2.0 : 1.0) * pw;    // C(m, i), m <= 2
                s = fma(w, g[i], s);
                pw *= -p2;
            }
            return s;
        };
        double s1a = 0.0, s1b = 0.0, s2a = 0.0, s2b = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            const double y = expand(a, G0, G1);
            s1a = fma(Pa[a], y, s1a);
            s1b = fma(Pb[a], y, s1b);
        }
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
            const double y = expand(a, K0, K1);
            s2a = fma(Qa[a], y, s2a);
            s2b = fma(Qb[a], y, s2b);
        }
        const double f = K.cd * invh;
        Ja += f * (gI * s1a - invh * s2a);
        Jb += f * (gI * s1b - invh * s2b);
    }
}

template <int DEG, int ORDER>
__global__ __launch_bounds__(256) void adjoint_kernel(const KArgs K, double invh, int64_t N,
                                                      const double *__restrict__ px, const double *__restrict__ py,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                      const double *__restrict__ tri,
                                                      const double *__restrict__ nodal,
                                                      const double *__restrict__ gI, const double *__restrict__ gX,
                                                      const double *__restrict__ gY, double *__restrict__ dpx,
                                                      double *__restrict__ dpy, double *__restrict__ pair_grad) {
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
    constexpr int NM = NN;                        // monomials of degree <= ORDER
    constexpr int NG = 6 + NN;
    const int lane = threadIdx.x & 63;
    const int64_t p0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
    if (p0 >= N) return;
    const int64_t pid = p0 + lane;
    const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
    const int64_t q_end = min(max(off[plast], (int64_t)0), P);
    const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
    const int64_t my_end = pid < N ? min(max(off[pid + 1], my_off), q_end) : q_end;
    const int64_t q_begin = __shfl(my_off, 0);
    double accX = 0.0, accY = 0.0;
    for (int64_t base = q_begin; base < q_end; base += 64) {
        const int64_t q = base + lane;
        const int64_t qq = q < q_end ? q : q_end - 1;
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
            if (lo + step < 64 && om <= qq) lo += step;
        }
        const int owner = lo;
        const int64_t ip = p0 + owner < N ? p0 + owner : N - 1;
        double vx = 0.0, vy = 0.0;
        if (q < q_end) {
            const int32_t t = tri_idx[q];
            double grad[NG];
#pragma unroll
            for (int k = 0; k < NG; ++k) grad[k] = 0.0;
            if (t >= 0 && t < T) {
                const double x = px[ip], y = py[ip];
                const double cI = gI[ip], cX = gX[ip], cY = gY[ip];
                double v[6], A[10];
#pragma unroll
                for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
#pragma unroll
                for (int k = 0; k < 10; ++k) A[k] = k < NN ? nodal[k * T + t] : 0.0;
                double ax[3], ay[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ax[i] = (v[2 * i] - x) * invh;
                    ay[i] = (v[2 * i + 1] - y) * invh;
                }
                const double area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
                if (area2 != 0.0) {
                    // field about the particle
                    double rec[kRecDoubles], c[10];
                    prepare_record<ORDER, double>(v, A, invh, rec);
                    taylor_shift<ORDER, double>(rec + 6, ax[0], ay[0], c);
                    // moments of the monomials about the particle, in one pass
                    double mom[NM];
                    // the cubic-field degree-11 variant keeps its edge loop rolled, like
                    // the forward kernel's: fully unrolled, that instantiation produced
                    // wrong moments (checked against the oracle in the tests) while
                    // the rolled form is correct
                    pair_dual<DEG, ORDER, (ORDER >= 2 && DEG > 8) ? 1 : 3>(K, ax, ay, area2, invh, cI, cX, cY, mom);
                    // nodal values: the moments carried back through the
                    // shift to the particle and the field preparation
                    {
                        double ge[10], gA[10];
                        taylor_shift_T<ORDER, double>(mom, ax[0], ay[0], ge);
                        prepare_record_T<ORDER, double>(v, ge, invh, gA);
#pragma unroll
                        for (int n = 0; n < NN; ++n) grad[6 + n] = gA[n];
                    }
                    // vertices, field part: -lambda_k dA/dx_alpha (ORDER >= 1)
                    if (ORDER >= 1) {
                        const double q1x = ax[1] - ax[0], q1y = ay[1] - ay[0];
                        const double q2x = ax[2] - ax[0], q2y = ay[2] - ay[0];
                        const double id = 1.0 / area2;
                        const double l1x = q2y * id, l1y = -q2x * id, l2x = -q1y * id, l2y = q1x * id;
                        const double lx[3] = {-(l1x + l2x), l1x, l2x};
                        const double ly[3] = {-(l1y + l2y), l1y, l2y};
                        // gradient of A in xi (units of h)
                        double dxA[10], dyA[10];
#pragma unroll
                        for (int k = 0; k < 10; ++k) dxA[k] = dyA[k] = 0.0;
#pragma unroll
                        for (int m = 1; m <= ORDER; ++m)
#pragma unroll
                            for (int j = 0; j <= m; ++j) {
                                const int i = m - j;
                                if (i > 0) dxA[pidx(i - 1, j)] += i * c[pidx(i, j)];
                                if (j > 0) dyA[pidx(i, j - 1)] += j * c[pidx(i, j)];
                            }
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            // lambda_k about the particle: 1 at vertex k, 0 at the others
                            const double l0 = (k == 0 ? 1.0 : 0.0) - lx[k] * ax[0] - ly[k] * ay[0];
                            double bx[10], by[10];
                            mul_affine<double>(dxA, l0, lx[k], ly[k], bx);
                            mul_affine<double>(dyA, l0, lx[k], ly[k], by);
                            double sx = 0.0, sy = 0.0;
#pragma unroll
                            for (int j = 0; j < NM; ++j) {
                                sx += bx[j] * mom[j];
                                sy += by[j] * mom[j];
                            }
                            grad[2 * k] -= invh * sx;
                            grad[2 * k + 1] -= invh * sy;
                        }
                    }
                    // vertices, boundary part
                    const double so = area2 > 0.0 ? 1.0 : -1.0;
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        const int f = e == 2 ? 0 : e + 1;
                        const double Lx = ax[f] - ax[e], Ly = ay[f] - ay[e];
                        const double len2 = Lx * Lx + Ly * Ly;
                        if (len2 == 0.0) continue;
                        const double len = sqrt(len2), ilen = 1.0 / len;
                        const double tx = Lx * ilen, ty = Ly * ilen;
                        const double sd = ax[e] * ty - ay[e] * tx;
                        const double pe = fabs(sd);
                        const double nx = sd > 0.0 ? ty : -ty, ny = sd > 0.0 ? -tx : tx;
                        const double ya = -ax[e] * ny + ay[e] * nx, yb = -ax[f] * ny + ay[f] * nx;
                        double Je, Jf;
                        edge_line<DEG, ORDER>(K, pe, ya, yb, nx, ny, c, cI, cX, cY, invh, Je, Jf);
                        const double ox = so * ty, oy = -so * tx;      // outward unit normal
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            if (k == e) {
                                grad[2 * k] += Je * ox;
                                grad[2 * k + 1] += Je * oy;
                            }
                            if (k == f) {
                                grad[2 * k] += Jf * ox;
                                grad[2 * k + 1] += Jf * oy;
                            }
                        }
                    }
                }
            }
            vx = -(grad[0] + grad[2] + grad[4]);
            vy = -(grad[1] + grad[3] + grad[5]);
            double *o = pair_grad + q * NG;
#pragma unroll
            for (int k = 0; k < NG; ++k) o[k] = grad[k];
        }
        // segmented scan over owners (pairs of a particle are contiguous)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double ux = __shfl_up(vx, d), uy = __shfl_up(vy, d);
            const int uo = __shfl_up(owner, d);
            if (lane >= d && uo == owner) {
                vx += ux;
                vy += uy;
            }
        }
        const int64_t s0 = my_off > base ? my_off : base;
        const int64_t s1 = my_end < base + 64 ? my_end : base + 64;
        const int src = s1 > s0 ? (int)(s1 - 1 - base) : 0;
        const double rx = __shfl(vx, src), ry = __shfl(vy, src);
        if (s1 > s0) {
            accX += rx;
            accY += ry;
        }
    }
    if (pid < N) {
        dpx[pid] = accX;
        dpy[pid] = accY;
    }
}

// start of every triangle's run in the triangle-sorted pair order
__global__ void tri_starts(int64_t P, int64_t T, const uint32_t *__restrict__ sorted_tri, int64_t *__restrict__ start) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T) return;
    int64_t lo = 0, hi = P;     // first index with sorted_tri[i] >= t
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)sorted_tri[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    start[t] = lo;
}

// Per-triangle sums of the per-pair gradients, in pair order: 16 lanes per
// triangle, lane k summing component k (the NG <= 16 components of a pair are
// contiguous, so the lanes read one pair's row together).
template <int NG>
__global__ __launch_bounds__(256) void tri_reduce(int64_t T, int n_nodes, const int64_t *__restrict__ start,
                                                  const int32_t *__restrict__ perm,
                                                  const double *__restrict__ pair_grad, double *__restrict__ dtri,
                                                  double *__restrict__ dnodal) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = g >> 4;
    const int k = (int)(g & 15);
    if (t >= T) return;
    double acc = 0.0;
    if (k < NG) {
        const int64_t i0 = start[t], i1 = start[t + 1];
        int64_t i = i0;
        // four pairs' loads in flight, added in pair order
        for (; i + 4 <= i1; i += 4) {
            const int32_t a = perm[i], b = perm[i + 1], c = perm[i + 2], d = perm[i + 3];
            const double ga = pair_grad[(int64_t)a * NG + k], gb = pair_grad[(int64_t)b * NG + k];
            const double gc = pair_grad[(int64_t)c * NG + k], gd = pair_grad[(int64_t)d * NG + k];
            acc += ga;
            acc += gb;
            acc += gc;
            acc += gd;
        }
        for (; i < i1; ++i) acc += pair_grad[(int64_t)perm[i] * NG + k];
    }
    if (k < 6) dtri[k * T + t] = acc;
    else if (k < 6 + n_nodes) dnodal[(k - 6) * T + t] = acc;
}

// Sort keys: the triangle index, or T for an index outside [0, T) (such pairs
// contribute nothing and sort after every triangle's run).
__global__ void sort_keys(int64_t P, int64_t T, const int32_t *__restrict__ tri_idx, uint32_t *__restrict__ key,
                          int32_t *__restrict__ iota) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int32_t t = tri_idx[i];
    key[i] = (t >= 0 && t < T) ? (uint32_t)t : (uint32_t)T;
    iota[i] = (int32_t)i;
}

template <int ORDER>
void launch_adj_deg(int deg, const KArgs &K, double invh, int64_t N, const double *px, const double *py,
                    const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T, const double *tri,
                    const double *nodal, const double *gI, const double *gX, const double *gY, double *dpx,
                    double *dpy, double *pair_grad, hipStream_t s) {
    const unsigned blocks = (unsigned)(((N + 63) / 64 + 3) / 4);
#define SPHBI_ADJ(DG)                                                                                            \
    hipLaunchKernelGGL((adjoint_kernel<DG, ORDER>), dim3(blocks), dim3(256), 0, s, K, invh, N, px, py, off,    \
                       tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy, pair_grad)
    if (deg <= 3) SPHBI_ADJ(3);
    else if (deg <= 5) SPHBI_ADJ(5);
    else if (deg <= 8) SPHBI_ADJ(8);
    else SPHBI_ADJ(11);
#undef SPHBI_ADJ
}

}  // namespace

size_t backward_workspace(int64_t T, int64_t P, int n_nodes) {
    const size_t NG = 6 + (size_t)n_nodes;
    size_t tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, (int)(P > 0 ? P : 1));
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    o += al((size_t)(P > 0 ? P : 1) * NG * sizeof(double));      // per-pair gradients
    o += 4 * al((size_t)(P > 0 ? P : 1) * sizeof(int32_t));       // keys, sorted keys, iota, permutation
    o += al((size_t)(T + 1) * sizeof(int64_t));                   // triangle starts
    o += al(tmp);
    return o;
}

int launch_backward(int order, int deg, const KArgs &K, double h, int64_t N, const double *px, const double *py,
                    const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T, const double *tri,
                    const double *nodal, const double *gI, const double *gX, const double *gY, double *dpx,
                    double *dpy, double *dtri, double *dnodal, void *ws, hipStream_t s) {
    const int NN = order == 0 ? 1 : (order == 1 ? 3 : 10);
    const size_t NG = 6 + (size_t)NN;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *w = (char *)ws;
    const int64_t Pn = P > 0 ? P : 1;
    double *pair_grad = (double *)w;
    w += al((size_t)Pn * NG * sizeof(double));
    uint32_t *keys_in = (uint32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    uint32_t *keys = (uint32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    int32_t *iota = (int32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    int32_t *perm = (int32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    int64_t *start = (int64_t *)w;
    w += al((size_t)(T + 1) * sizeof(int64_t));
    size_t tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, (int)Pn);
    const double invh = 1.0 / h;
    if (N > 0) {
        if (order == 0)
            launch_adj_deg<0>(deg, K, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy, pair_grad, s);
        else if (order == 1)
            launch_adj_deg<1>(deg, K, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy, pair_grad, s);
        else
            launch_adj_deg<3>(deg, K, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy, pair_grad, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("adjoint launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    if (T == 0) return SPHBI_OK;
    if (P > 0) {
        hipLaunchKernelGGL(sort_keys, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, T, tri_idx, keys_in, iota);
        int bits = 1;                                  // keys are in [0, T]
        while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)T) ++bits;
        e = hipcub::DeviceRadixSort::SortPairs(w, tmp, keys_in, keys, iota, perm, (int)P, 0, bits, s);
        if (e != hipSuccess) { set_error("pair sort: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    }
    hipLaunchKernelGGL(tri_starts, dim3((unsigned)((T + 1 + 255) / 256)), dim3(256), 0, s, P, T, keys, start);
    const unsigned tb = (unsigned)((T * 16 + 255) / 256);
    if (NN == 1) hipLaunchKernelGGL(tri_reduce<7>, dim3(tb), dim3(256), 0, s, T, 1, start, perm, pair_grad, dtri, dnodal);
    else if (NN == 3) hipLaunchKernelGGL(tri_reduce<9>, dim3(tb), dim3(256), 0, s, T, 3, start, perm, pair_grad, dtri, dnodal);
    else hipLaunchKernelGGL(tri_reduce<16>, dim3(tb), dim3(256), 0, s, T, 10, start, perm, pair_grad, dtri, dnodal);
    e = hipGetLastError();
    if (e != hipSuccess) { set_error("adjoint reduction: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
