// Forward integrals: the field-preparation kernel (per-triangle records) and
// the launch of the pair kernels of forward_pair.h for plain fields.

#include <math.h>

#include "forward_pair.h"

namespace sphbi {
namespace {

template <int ORDER>
__global__ __launch_bounds__(256) void prepare_kernel(int64_t T, const double *__restrict__ tri,
                                                      const double *__restrict__ nodal, double invh,
                                                      double *__restrict__ rec,
                                                      unsigned long long *__restrict__ count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0 && count) {                // the refinement counter of the next forward pass
        count[0] = 0;
        count[1] = 0;                     // and the refinement pass's window counter
    }
    if (t >= T) return;
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
    double v[6], A[10];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
#pragma unroll
    for (int k = 0; k < 10; ++k) A[k] = k < NN ? nodal[k * T + t] : 0.0;
    double r[kRecDoubles];
    prepare_record<ORDER, double>(v, A, invh, r);
    double *o = rec + t * kRecDoubles;
#pragma unroll
    for (int k = 0; k < kRecDoubles; ++k) o[k] = r[k];
}

template <bool MIXED>
void launch_fwd_order(int order, int deg, const KArgs &K, const FwdArgs &a, hipStream_t s) {
    if (order == 0) launch_fwd_deg<0, MIXED>(deg, K, a, s);
    else if (order == 1) launch_fwd_deg<1, MIXED>(deg, K, a, s);
    else launch_fwd_deg<3, MIXED>(deg, K, a, s);
}

}  // namespace

int launch_prepare(int order, int64_t T, const double *tri, const double *nodal, double h, double *rec,
                   hipStream_t s, unsigned long long *count) {
    if (T == 0) return SPHBI_OK;
    const unsigned blocks = (unsigned)((T + 255) / 256);
    const double invh = 1.0 / h;
    if (order == 0)
        hipLaunchKernelGGL(prepare_kernel<0>, dim3(blocks), dim3(256), 0, s, T, tri, nodal, invh, rec, count);
    else if (order == 1)
        hipLaunchKernelGGL(prepare_kernel<1>, dim3(blocks), dim3(256), 0, s, T, tri, nodal, invh, rec, count);
    else hipLaunchKernelGGL(prepare_kernel<3>, dim3(blocks), dim3(256), 0, s, T, tri, nodal, invh, rec, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("prepare launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int launch_forward(int order, int deg, int precision, double tau_edge, const KArgs &K, const RefineGate &gate,
                   double h, int64_t N, const double *px, const double *py, const int64_t *offsets,
                   const int32_t *tri_idx, int64_t P, int64_t T, const double *rec, double *I, double *Gx, double *Gy,
                   double *per_pair, hipStream_t s, uint8_t *status) {
    if (N == 0) return SPHBI_OK;
    const FwdArgs a{tau_edge, 1.0 / h, N, px, py, offsets, tri_idx, rec, I, Gx, Gy, per_pair, P, T, nullptr, nullptr,
                    gate, status};
    if (precision == SPHBI_MIXED) launch_fwd_order<true>(order, deg, K, a, s);
    else launch_fwd_order<false>(order, deg, K, a, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("forward launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
