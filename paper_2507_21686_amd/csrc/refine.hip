// Double-double evaluation of ill-conditioned pairs (the forward integrals of
// Sec. 2-5 with every step in double-double; see ddmath.h for why a pair can
// need it).
//
// refine_kernel evaluates the selected pairs -- all pairs, or those whose
// conditioning gate fires (refine.h) -- from the triangles' world coordinates
// and nodal values in double-double, rounds each to FP64 and sums them per
// particle in pair order.  In the gated mode the forward kernel has left
// these pairs out of its sums and the refined ones are added to its outputs;
// in the all-pairs mode the outputs are written here alone.  A launch that
// finds the forward pass's counter at zero returns at once.

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

// One wavefront owns 64 consecutive particles (a grid of a few blocks per
// compute unit strides over the groups).  It sweeps its particles' pairs 64
// at a time, one pair per lane, and appends the pairs to refine (every pair
// with a valid triangle in the all-pairs mode, else those whose gate fires)
// to a list in LDS, in pair order; whenever the list is full, and at the end,
// the list is evaluated one pair per lane and every particle lane adds the
// results of its own pairs in list order.  The lanes therefore run the costly
// double-double pairs densely, whatever the pairs' distribution over the
// particles, and the sums stay in pair order (deterministic).
constexpr int kRefList = 128;

template <int DEG, int ORDER>
__global__ __launch_bounds__(64) void refine_kernel(const KArgsDD K, RefineGate gate, bool all, double invh,
                                                     int64_t N, const double *__restrict__ px,
                                                     const double *__restrict__ py, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                     const double *__restrict__ tri,
                                                     const double *__restrict__ nodal, double *__restrict__ I,
                                                     double *__restrict__ Gx, double *__restrict__ Gy,
                                                     double *__restrict__ per_pair, uint8_t *__restrict__ status) {
    __shared__ int64_t s_q[kRefList];
    __shared__ uint8_t s_own[kRefList];
    __shared__ double s_res[kRefList][3];
    if (!all && *gate.count == 0) return;       // the forward pass left out no pair
    const int lane = threadIdx.x;
    for (int64_t p0 = (int64_t)blockIdx.x * 64; p0 < N; p0 += (int64_t)gridDim.x * 64) {
        const int64_t pid = p0 + lane;
        const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
        // the forward kernels' clamping of the CSR range
        const int64_t q_end = min(max(off[plast], (int64_t)0), P);
        const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
        const int64_t q_begin = __shfl(my_off, 0);
        double aI = 0.0, aX = 0.0, aY = 0.0;
        bool any = false;
        int n_list = 0;
        // evaluates the listed pairs and adds them to their particles
        auto flush = [&]() {
            for (int j = lane; j < n_list; j += 64) {
                const int64_t q = s_q[j];
                const int64_t ip = p0 + s_own[j];
                double vI, vX, vY;
                pair_dd<DEG, ORDER>(K, px[ip], py[ip], invh, tri, nodal, T, tri_idx[q], vI, vX, vY);
                s_res[j][0] = vI;
                s_res[j][1] = vX;
                s_res[j][2] = vY;
                if (per_pair) {
                    per_pair[q] = vI;
                    per_pair[P + q] = vX;
                    per_pair[2 * P + q] = vY;
                }
                if (status) status[q] = !(isfinite(vI) && isfinite(vX) && isfinite(vY));
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int j = 0; j < n_list; ++j)
                if (s_own[j] == lane) {
                    aI += s_res[j][0];
                    aX += s_res[j][1];
                    aY += s_res[j][2];
                    any = true;
                }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            n_list = 0;
        };
        for (int64_t base = q_begin; base < q_end; base += 64) {
            const int64_t q = base + lane;
            const int64_t qq = q < q_end ? q : q_end - 1;
            int lo = 0;                                // owner lane (the forward kernels' search)
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
                if (lo + step < 64 && om <= qq) lo += step;
            }
            bool take = false;
            if (q < q_end) {
                const int32_t t = tri_idx[q];
                if (t >= 0 && t < T) {
                    if (all) {
                        take = true;
                    } else {
                        const int64_t ip = p0 + lo;
                        double ax[3], ay[3];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            ax[k] = (tri[(2 * k) * T + t] - px[ip]) * invh;
                            ay[k] = (tri[(2 * k + 1) * T + t] - py[ip]) * invh;
                        }
                        take = gate.fires(ax, ay);
                    }
                } else if (all) {
                    if (per_pair) per_pair[q] = per_pair[P + q] = per_pair[2 * P + q] = 0.0;
                    if (status) status[q] = 0;
                }
            }
            const uint64_t mask = __ballot(take);
            const int cnt = __popcll(mask);
            if (cnt == 0) continue;
            if (n_list + cnt > kRefList) flush();
            if (take) {
                const int slot = n_list + __popcll(mask & ((1ull << lane) - 1));
                s_q[slot] = q;
                s_own[slot] = (uint8_t)lo;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            n_list += cnt;
        }
        if (n_list) flush();
        if (pid < N) {
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
    }
}

template <int ORDER>
void launch_refine_order(int deg, const KArgsDD &K, const RefineGate &g, bool all, double invh, int64_t N,
                         const double *px, const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P,
                         int64_t T, const double *tri, const double *nodal, double *I, double *Gx, double *Gy,
                         double *per_pair, hipStream_t s, uint8_t *status) {
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
                       tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, status)
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
                  double *per_pair, hipStream_t s, uint8_t *status) {
    if (N == 0) return SPHBI_OK;
    const KArgsDD D = make_kargs_dd(K);
    const double invh = 1.0 / h;
    if (order == 0)
        launch_refine_order<0>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s, status);
    else if (order == 1)
        launch_refine_order<1>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status);
    else
        launch_refine_order<3>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("refine launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
