// Adjoint pair kernel: given cotangents (gI, gGx, gGy) per particle,
// gradients with respect to particle positions, triangle vertices and nodal
// field values.
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
//     radial terms H_c = int rho^(c-1) dy and powers of rho that the closed
//     form of the same edge forms anyway (LineSums, taken in pair_dual).
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
// segmented wave scan; per-pair triangle gradients go to a buffer that the
// reduction in adjoint.hip sums per triangle.
//
// Two translation units instantiate it: adjoint.hip (constant and cubic
// fields, plain FP64 constants) and adjoint_linear.hip (linear field,
// constants as scalar-register operands, which is faster there).  The
// anonymous namespace keeps each unit's copy its own.

#pragma once

#include <math.h>

#include <type_traits>

#include "internal.h"
#include "pairmath.h"

namespace sphbi {
namespace {

template <int DEG, int ORDER, bool MIXED, typename KA>
__global__ __launch_bounds__(64) void adjoint_kernel(const KA K, double tau, double invh, int64_t N,
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
                    // moments of the monomials about the particle and the
                    // boundary part of the vertex gradients, in one pass
                    double mom[NM], gv[6];
                    if (MIXED)
                        pair_dual<DEG, ORDER, 3, MixedMath, KA>(K, ax, ay, area2, invh, cI, cX, cY, c, mom, gv,
                                                            MixedMath{false, ORDER >= 2}, tau);
                    else pair_dual<DEG, ORDER, 3, ExactMath, KA>(K, ax, ay, area2, invh, cI, cX, cY, c, mom, gv);
#pragma unroll
                    for (int k = 0; k < 6; ++k) grad[k] = gv[k];
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

template <int ORDER, bool MIXED>
void launch_adj_deg(int deg, const KArgs &K, double tau, double invh, int64_t N, const double *px, const double *py,
                    const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T, const double *tri,
                    const double *nodal, const double *gI, const double *gX, const double *gY, double *dpx,
                    double *dpy, double *pair_grad, hipStream_t s) {
    const unsigned blocks = (unsigned)((N + 63) / 64);
#define SPHBI_ADJ(DG)                                                                                         \
    with_zero_pattern<DG>(K, [&](const auto &KZ) {                                                           \
        using KA = std::decay_t<decltype(KZ)>;                                                              \
        hipLaunchKernelGGL((adjoint_kernel<DG, ORDER, MIXED, KA>), dim3(blocks), dim3(64), 0, s, KZ, tau, invh, N, \
                           px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy, pair_grad);            \
    })
    if (deg <= 3) SPHBI_ADJ(3);
    else if (deg <= 5) SPHBI_ADJ(5);
    else if (deg <= 8) SPHBI_ADJ(8);
    else SPHBI_ADJ(11);
#undef SPHBI_ADJ
}

}  // namespace
}  // namespace sphbi
