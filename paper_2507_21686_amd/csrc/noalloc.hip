// sphbi_integrate_noalloc: the forward integrals with the per-triangle field
// records kept in a fixed device array of this library instead of a
// caller-supplied workspace, for callers that cannot allocate.
//
// The array lives for the whole process, one copy per GPU.  Host code never
// uses its symbol as an address: the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress (that device current)
// and kept in a per-device table.

#include <mutex>

#include "internal.h"

namespace sphbi {
namespace {

constexpr int64_t kNoAllocMaxT = SPHBI_NOALLOC_MAX_TRIANGLES;
constexpr int kMaxDevices = 64;

// Field records of at most kNoAllocMaxT triangles (16 MiB), the refinement
// pass's counters behind them and its double-double records (32 MiB): the
// layout of sphbi_integrate's workspace.
constexpr size_t kScratchDoubles = kNoAllocMaxT * kRecDoubles + 32 + 2 * kNoAllocMaxT * kRecDoubles;
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_ptr(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_error("hipGetDevice: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    if (dev < 0 || dev >= kMaxDevices) { set_error("device %d out of range", dev); return SPHBI_EUNSUPPORTED; }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return SPHBI_EDEVICE;
        }
        g_ptr[dev] = p;
    }
    *out = (double *)g_ptr[dev];
    return SPHBI_OK;
}

}  // namespace
}  // namespace sphbi

using namespace sphbi;

extern "C" int sphbi_integrate_noalloc(const sphbi_kernel *kernel, const sphbi_opts *opts, double h,
                                       int32_t n_nodes, int64_t N, const double *px, const double *py, int64_t T,
                                       const double *tri, const double *nodal, const int64_t *offsets,
                                       const int32_t *tri_idx, int64_t n_pairs, double *I, double *Gx, double *Gy,
                                       double *per_pair, void *stream) {
    if (T > kNoAllocMaxT) {
        set_error("sphbi_integrate_noalloc: %lld triangles exceed its fixed record array of %lld",
                  (long long)T, (long long)kNoAllocMaxT);
        return SPHBI_EUNSUPPORTED;
    }
    int rc = check_integrate_args(kernel, opts, h, n_nodes, N, px, py, T, tri, nodal, offsets, tri_idx, n_pairs, I,
                                  Gx, Gy, per_pair);
    if (rc) return rc;
    if (N == 0) return SPHBI_OK;
    double *rec = nullptr;
    rc = scratch_ptr(&rec);
    if (rc) return rc;
    const size_t bytes = kScratchDoubles * sizeof(double);
    // (kNoAllocMaxT records take a multiple of 256 bytes, as records_bytes rounds to)
    static_assert((kNoAllocMaxT * kRecDoubles * sizeof(double)) % 256 == 0 &&
                      kScratchDoubles * sizeof(double) >= 3 * kNoAllocMaxT * kRecDoubles * sizeof(double) + 256,
                  "records, counters and double-double records must fit");
    return integrate_run(kernel, opts, h, n_nodes, N, px, py, T, tri, nodal, rec, bytes, offsets, tri_idx, n_pairs, I,
                         Gx, Gy, per_pair, stream);
}
