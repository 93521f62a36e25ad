// Measurement probe: the FP64 vector FMA rate of the device, measured on the
// same GPU as the kernels whose rates are compared with it.  Every lane runs
// kChains independent chains of dependent fused multiply-adds, so that a
// wavefront always has an FMA ready to issue, with eight waves per SIMD.

#include "internal.h"

namespace sphbi {
namespace {

constexpr int kChains = 8;
constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void fma_probe_kernel(int64_t iters, double *__restrict__ sink) {
    double a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = 1.0 + 1e-3 * (double)(threadIdx.x + c);
    const double m = 0.9999999999999, q = 1e-13;
#pragma unroll 4
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = fma(a[c], m, q);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    if (s == -1.0) sink[0] = s;       // never true (the chains stay near 1): keeps them live
}

}  // namespace
}  // namespace sphbi

using namespace sphbi;

extern "C" int sphbi_probe_fp64_fma(int64_t iters, double *sink, double *flops, void *stream) {
    if (iters < 1 || iters > ((int64_t)1 << 24) || !sink || !flops) {
        set_error("sphbi_probe_fp64_fma: iters in [1, 2^24], sink and flops required");
        return SPHBI_EINVAL;
    }
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) {
        set_error("sphbi_probe_fp64_fma: no device attributes");
        return SPHBI_EDEVICE;
    }
    // eight waves per SIMD: 8 x 4 SIMDs x 64 lanes per compute unit
    const int64_t blocks = (int64_t)n_cu * 8;
    hipLaunchKernelGGL(fma_probe_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0, (hipStream_t)stream, iters,
                       sink);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("probe launch: %s", hipGetErrorString(e));
        return SPHBI_EDEVICE;
    }
    *flops = 2.0 * (double)kChains * (double)iters * (double)(blocks * kProbeThreads);
    return SPHBI_OK;
}
