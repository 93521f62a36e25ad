// Adjoint of the forward integrals: given cotangents (gI, gGx, gGy) per
// particle, gradients with respect to particle positions, triangle vertices
// and nodal field values.
//
// Nothing from the forward pass is stored: every pair recomputes its field
// record and its clipping/decomposition.  Derivatives with respect to the six
// vertex coordinates come from a forward-mode dual-number evaluation of the
// same closed forms (pairmath.h), including the dependence of the field
// polynomial on the vertices.  The particle gradient follows from
// translation invariance (moving particle and triangle together changes
// nothing): d/dx = -(d/dv0 + d/dv1 + d/dv2).  The integrals are linear in
// the nodal values, so d/dA_n is the pair evaluated with the unit field e_n.
//
// Particle gradients are summed per particle with the forward kernel's
// segmented wave scan.  Per-pair triangle gradients go to a buffer and are
// summed per triangle in pair order through a stable sort by triangle index,
// so the whole adjoint is deterministic.

#include <math.h>

#include <hipcub/hipcub.hpp>

#include "dual.h"
#include "internal.h"
#include "pairmath.h"

namespace sphbi {
namespace {

using D6 = Dual<6>;

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
                // vertices: six dual directions
                {
                    D6 vd[6], Ad[10], rec[kRecDoubles];
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        vd[k] = D6(v[k]);
                        vd[k].d[k] = 1.0;
                    }
#pragma unroll
                    for (int k = 0; k < 10; ++k) Ad[k] = D6(A[k]);
                    prepare_record<ORDER, D6>(vd, Ad, invh, rec);
                    D6 oI, oX, oY;
                    pair_fwd<DEG, ORDER, D6>(K, ExactMath(), 0.0, D6(x), D6(y), invh, rec, oI, oX, oY);
#pragma unroll
                    for (int k = 0; k < 6; ++k) grad[k] = cI * oI.d[k] + cX * oX.d[k] + cY * oY.d[k];
                }
                // nodal values: the integrals are linear in them
#pragma unroll 1
                for (int n = 0; n < NN; ++n) {
                    double Au[10], rec[kRecDoubles];
#pragma unroll
                    for (int k = 0; k < 10; ++k) Au[k] = k == n ? 1.0 : 0.0;
                    prepare_record<ORDER, double>(v, Au, invh, rec);
                    double oI, oX, oY;
                    pair_fwd<DEG, ORDER, double>(K, ExactMath(), 0.0, x, y, invh, rec, oI, oX, oY);
                    grad[6 + n] = cI * oI + cX * oX + cY * oY;
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
__global__ void tri_starts(int64_t P, int64_t T, const int32_t *__restrict__ sorted_tri, int64_t *__restrict__ start) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T) return;
    int64_t lo = 0, hi = P;     // first index with sorted_tri[i] >= t
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sorted_tri[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    start[t] = lo;
}

__global__ void iota_i32(int64_t P, int32_t *__restrict__ a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) a[i] = (int32_t)i;
}

template <int NG>
__global__ void tri_reduce(int64_t T, int n_nodes, const int64_t *__restrict__ start, const int32_t *__restrict__ perm,
                           const double *__restrict__ pair_grad, double *__restrict__ dtri,
                           double *__restrict__ dnodal) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double acc[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) acc[k] = 0.0;
    for (int64_t i = start[t]; i < start[t + 1]; ++i) {
        const double *g = pair_grad + (int64_t)perm[i] * NG;
#pragma unroll
        for (int k = 0; k < NG; ++k) acc[k] += g[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) dtri[k * T + t] = acc[k];
    for (int n = 0; n < n_nodes; ++n) dnodal[n * T + t] = acc[6 + n];
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
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const int32_t *)nullptr, (int32_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, (int)(P > 0 ? P : 1));
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    o += al((size_t)(P > 0 ? P : 1) * NG * sizeof(double));      // per-pair gradients
    o += 3 * al((size_t)(P > 0 ? P : 1) * sizeof(int32_t));       // iota, sorted keys, permutation
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
    int32_t *iota = (int32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    int32_t *keys = (int32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    int32_t *perm = (int32_t *)w;
    w += al((size_t)Pn * sizeof(int32_t));
    int64_t *start = (int64_t *)w;
    w += al((size_t)(T + 1) * sizeof(int64_t));
    size_t tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const int32_t *)nullptr, (int32_t *)nullptr,
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
        hipLaunchKernelGGL(iota_i32, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, iota);
        e = hipcub::DeviceRadixSort::SortPairs(w, tmp, tri_idx, keys, iota, perm, (int)P, 0, 32, s);
        if (e != hipSuccess) { set_error("pair sort: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    }
    hipLaunchKernelGGL(tri_starts, dim3((unsigned)((T + 1 + 255) / 256)), dim3(256), 0, s, P, T, keys, start);
    const unsigned tb = (unsigned)((T + 255) / 256);
    if (NN == 1) hipLaunchKernelGGL(tri_reduce<7>, dim3(tb), dim3(256), 0, s, T, 1, start, perm, pair_grad, dtri, dnodal);
    else if (NN == 3) hipLaunchKernelGGL(tri_reduce<9>, dim3(tb), dim3(256), 0, s, T, 3, start, perm, pair_grad, dtri, dnodal);
    else hipLaunchKernelGGL(tri_reduce<16>, dim3(tb), dim3(256), 0, s, T, 10, start, perm, pair_grad, dtri, dnodal);
    e = hipGetLastError();
    if (e != hipSuccess) { set_error("adjoint reduction: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
