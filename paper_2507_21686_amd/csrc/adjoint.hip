// Adjoint of the forward integrals: given cotangents (gI, gGx, gGy) per
// particle, gradients with respect to particle positions, triangle vertices
// and nodal field values.  The pair kernel (adjoint_pair.h) writes particle
// gradients directly and per-pair triangle gradients to a buffer; here they
// are summed per triangle in pair order through a stable sort by triangle
// index, so the whole adjoint is deterministic.

#include <math.h>

#include <rocprim/device/device_radix_sort.hpp>

// plain FP64 constants in this unit (see sconst)
#define SPHBI_PLAIN_CONSTANTS 1

#include "adjoint_pair.h"

namespace sphbi {
namespace {

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

// Sort keys: the triangle index, or T for a pair that contributes nothing:
// an index outside [0, T), or a pair outside the particles' range
// [offsets[0], offsets[N]) of the CSR list, which the pair kernel does not
// visit (and whose gradient slots it leaves unwritten).  Such pairs sort
// after every triangle's run.
__global__ void sort_keys(int64_t P, int64_t T, int64_t N, const int64_t *__restrict__ off,
                          const int32_t *__restrict__ tri_idx, uint32_t *__restrict__ key,
                          int32_t *__restrict__ iota) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    // the pair kernel's own clamping of the range
    const int64_t hi = N > 0 ? min(max(off[N], (int64_t)0), P) : 0;
    const int64_t lo = N > 0 ? min(max(off[0], (int64_t)0), hi) : 0;
    const int32_t t = tri_idx[i];
    key[i] = (i >= lo && i < hi && t >= 0 && t < T) ? (uint32_t)t : (uint32_t)T;
    iota[i] = (int32_t)i;
}

}  // namespace

size_t backward_workspace(int64_t T, int64_t P, int n_nodes) {
    const size_t NG = 6 + (size_t)n_nodes;
    size_t tmp = 0;
    (void)rocprim::radix_sort_pairs(nullptr, tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                    (const int32_t *)nullptr, (int32_t *)nullptr, (size_t)(P > 0 ? P : 1));
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    o += al((size_t)(P > 0 ? P : 1) * NG * sizeof(double));      // per-pair gradients
    o += 4 * al((size_t)(P > 0 ? P : 1) * sizeof(int32_t));       // keys, sorted keys, iota, permutation
    o += al((size_t)(T + 1) * sizeof(int64_t));                   // triangle starts
    o += al(tmp);
    return o;
}

int launch_backward(int order, int deg, int precision, double tau, const KArgs &K, double h, int64_t N,
                    const double *px, const double *py,
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
    (void)rocprim::radix_sort_pairs(nullptr, tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                    (const int32_t *)nullptr, (int32_t *)nullptr, (size_t)Pn);
    const double invh = 1.0 / h;
    const bool mixed = precision == SPHBI_MIXED;
    if (N > 0) {
        if (order == 1)
            launch_adjoint_linear(deg, mixed, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx,
                                  dpy, pair_grad, s);
        else if (order == 0 && mixed)
            launch_adj_deg<0, true>(deg, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy,
                                    pair_grad, s);
        else if (order == 0)
            launch_adj_deg<0, false>(deg, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx,
                                     dpy, pair_grad, s);
        else if (mixed)
            launch_adj_deg<3, true>(deg, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy,
                                    pair_grad, s);
        else
            launch_adj_deg<3, false>(deg, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx,
                                     dpy, pair_grad, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("adjoint launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    if (T == 0) return SPHBI_OK;
    if (P > 0) {
        hipLaunchKernelGGL(sort_keys, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, T, N, off, tri_idx, keys_in,
                           iota);
        int bits = 1;                                  // keys are in [0, T]
        while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)T) ++bits;
        e = rocprim::radix_sort_pairs(w, tmp, keys_in, keys, iota, perm, (size_t)P, 0u, (unsigned)bits, s);
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
