// Double-double evaluation of ill-conditioned pairs (the forward integrals of
// Sec. 2-5 with every step in double-double; see ddmath.h for why a pair can
// need it).
//
// refine_kernel: one lane per particle, 64 particles per block, the blocks
// striding over the particles (a grid of at most a few blocks per compute
// unit, so that a launch with nothing to refine costs little).  A lane walks
// its particle's pairs in CSR order; every pair selected by the policy
// (all pairs, or those whose conditioning gate fires, see refine_gate) is
// evaluated from the triangle's world coordinates and nodal values in
// double-double, rounded to FP64, and summed in pair order.  In the gated
// mode the forward kernel has left these pairs out of its sums and the
// refined ones are added to its outputs; in the all-pairs mode the outputs
// are written here alone.

#include <math.h>
#include <string.h>

#include "refine.h"

namespace sphbi {
namespace {

// One pair in double-double: the field record of the triangle is rebuilt from
// the exact input doubles and the pair is evaluated by the same closed form
// as the FP64 kernels.
template <int DEG, int ORDER>
__device__ __noinline__ void pair_dd(const KArgsDD &K, double x, double y, double invh, const double *__restrict__ tri,
                                     const double *__restrict__ nodal, int64_t T, int64_t t, double &oI, double &oX,
                                     double &oY) {
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
    dd v[6], A[10];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = dd(tri[k * T + t]);
#pragma unroll
    for (int k = 0; k < 10; ++k) A[k] = dd(k < NN ? nodal[k * T + t] : 0.0);
    dd r[kRecDoubles];
    prepare_record<ORDER, dd>(v, A, invh, r);
    dd I, X, Y;
    pair_fwd<DEG, ORDER, dd, DDMath, 1>(K, DDMath(), 0.0, dd(x), dd(y), invh, r, I, X, Y);
    oI = (double)I;
    oX = (double)X;
    oY = (double)Y;
}

template <int DEG, int ORDER>
__device__ inline void refine_particle(const KArgsDD &K, const RefineGate &gate, bool all, double invh, int64_t N,
                                       int64_t pid, const double *__restrict__ px, const double *__restrict__ py,
                                       const int64_t *__restrict__ off, const int32_t *__restrict__ tri_idx,
                                       int64_t P, int64_t T, int64_t q_lo, int64_t q_end,
                                       const double *__restrict__ tri, const double *__restrict__ nodal,
                                       double *__restrict__ I, double *__restrict__ Gx, double *__restrict__ Gy,
                                       double *__restrict__ per_pair) {
    const int64_t my_off = min(max(off[pid], q_lo), q_end);
    const int64_t my_end = min(max(off[pid + 1], my_off), q_end);
    const double x = px[pid], y = py[pid];
    double aI = 0.0, aX = 0.0, aY = 0.0;
    bool any = false;
    for (int64_t q = my_off; q < my_end; ++q) {
        const int32_t t = tri_idx[q];
        if (t < 0 || t >= T) {
            if (all && per_pair) per_pair[q] = per_pair[P + q] = per_pair[2 * P + q] = 0.0;
            continue;
        }
        if (!all) {
            double ax[3], ay[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ax[k] = (tri[(2 * k) * T + t] - x) * invh;
                ay[k] = (tri[(2 * k + 1) * T + t] - y) * invh;
            }
            if (!gate.fires(ax, ay)) continue;
        }
        double vI, vX, vY;
        pair_dd<DEG, ORDER>(K, x, y, invh, tri, nodal, T, t, vI, vX, vY);
        if (per_pair) {
            per_pair[q] = vI;
            per_pair[P + q] = vX;
            per_pair[2 * P + q] = vY;
        }
        aI += vI;
        aX += vX;
        aY += vY;
        any = true;
    }
    if (all) {
        I[pid] = aI;
        Gx[pid] = aX;
        Gy[pid] = aY;
    } else if (any) {
        I[pid] += aI;
        Gx[pid] += aX;
        Gy[pid] += aY;
    }
}

template <int DEG, int ORDER>
__global__ __launch_bounds__(64) void refine_kernel(const KArgsDD K, RefineGate gate, bool all, double invh,
                                                     int64_t N, const double *__restrict__ px,
                                                     const double *__restrict__ py, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                     const double *__restrict__ tri,
                                                     const double *__restrict__ nodal, double *__restrict__ I,
                                                     double *__restrict__ Gx, double *__restrict__ Gy,
                                                     double *__restrict__ per_pair) {
    if (!all && *gate.count == 0) return;       // the forward pass left out no pair
    // the forward kernels' clamping of the CSR range
    const int64_t q_end = min(max(off[N], (int64_t)0), P);
    const int64_t q_lo = min(max(off[0], (int64_t)0), q_end);
    for (int64_t pid = (int64_t)blockIdx.x * 64 + threadIdx.x; pid < N; pid += (int64_t)gridDim.x * 64)
        refine_particle<DEG, ORDER>(K, gate, all, invh, N, pid, px, py, off, tri_idx, P, T, q_lo, q_end, tri, nodal, I,
                                    Gx, Gy, per_pair);
}

template <int ORDER>
void launch_refine_order(int deg, const KArgsDD &K, const RefineGate &g, bool all, double invh, int64_t N,
                         const double *px, const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P,
                         int64_t T, const double *tri, const double *nodal, double *I, double *Gx, double *Gy,
                         double *per_pair, hipStream_t s) {
    // a few waves per compute unit: enough to fill the chip when every pair
    // is refined (the kernel runs one wave per SIMD), little to launch when
    // none is
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 256;
    const int64_t want = (N + 63) / 64, cap = (int64_t)n_cu * 8;
    const unsigned blocks = (unsigned)(want < cap ? want : cap);
#define SPHBI_REF(DG)                                                                                          \
    hipLaunchKernelGGL((refine_kernel<DG, ORDER>), dim3(blocks), dim3(64), 0, s, K, g, all, invh, N, px, py, off, \
                       tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair)
    if (deg <= 3) SPHBI_REF(3);
    else if (deg <= 5) SPHBI_REF(5);
    else if (deg <= 8) SPHBI_REF(8);
    else SPHBI_REF(11);
#undef SPHBI_REF
}

}  // namespace

KArgsDD make_kargs_dd(const KArgs &K) {
    KArgsDD D;
    memset(&D, 0, sizeof(D));
    D.npieces = K.npieces;
    D.cd = K.cd;
    for (int p = 0; p < 2; ++p) {
        D.R[p] = K.R[p];
        D.iR[p] = K.iR[p];
        for (int k = 0; k <= kMaxDeg; ++k) D.b[p][k] = K.b[p][k];
        if (p >= K.npieces) continue;
        for (int m = 0; m <= kMaxOrder; ++m) {
            // sv = sum_k b_k R^(k+2+m) / (k+2+m), sw = sum_k k b_k R^(k+1+m) / (k+1+m)
            dd sv(0.0), sw(0.0), Rn(1.0);
            dd Rp[kMaxDeg + kMaxOrder + 3];
            for (int n = 0; n < kMaxDeg + kMaxOrder + 3; ++n) {
                Rp[n] = Rn;
                Rn = Rn * K.R[p];
            }
            for (int k = 0; k <= kMaxDeg; ++k) {
                const double b = K.b[p][k];
                if (b == 0.0) continue;
                sv = sv + (Rp[k + 2 + m] * b) * dd_recip(k + 2 + m);
                if (k >= 1) sw = sw + (Rp[k + 1 + m] * (b * (double)k)) * dd_recip(k + 1 + m);
            }
            D.sv[p][m] = sv;
            D.sw[p][m] = sw;
        }
    }
    return D;
}

int launch_refine(int order, int deg, const KArgs &K, const RefineGate &gate, bool all, double h, int64_t N,
                  const double *px, const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P,
                  int64_t T, const double *tri, const double *nodal, double *I, double *Gx, double *Gy,
                  double *per_pair, hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    const KArgsDD D = make_kargs_dd(K);
    const double invh = 1.0 / h;
    if (order == 0)
        launch_refine_order<0>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s);
    else if (order == 1)
        launch_refine_order<1>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s);
    else
        launch_refine_order<3>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("refine launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
