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

#include <algorithm>

#include "refine.h"

namespace sphbi {
namespace {

// The field record of triangle t in double-double, from the exact input
// doubles.
template <int ORDER>
__device__ inline void record_dd(double invh, const double *__restrict__ tri, const double *__restrict__ nodal,
                                 int64_t T, int64_t t, dd *r) {
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
    dd v[6], A[10];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = dd(tri[k * T + t]);
#pragma unroll
    for (int k = 0; k < 10; ++k) A[k] = dd(k < NN ? nodal[k * T + t] : 0.0);
    prepare_record<ORDER, dd>(v, A, invh, r);
}

// Every triangle's double-double record, once per call (stored as hi, lo
// pairs, kRecDoubles of them per triangle), so that the pairs of a triangle
// do not each rebuild it.  It pays only when the refinement kernel's waves
// evaluate several lists each: with fewer than dense_min refined pairs (one
// list per wave) every wave's time is the latency of one list, and building
// the records first would only add the latency of one record.  Both kernels
// read the forward pass's count and take the same decision.
template <int ORDER>
__global__ __launch_bounds__(256) void prepare_dd_kernel(RefineGate gate, bool all, unsigned long long dense_min,
                                                         double invh, int64_t T, const double *__restrict__ tri,
                                                         const double *__restrict__ nodal, double *__restrict__ rec_dd) {
    if (!all && *gate.count < dense_min) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    dd r[kRecDoubles];
    record_dd<ORDER>(invh, tri, nodal, T, t, r);
    double *o = rec_dd + t * 2 * kRecDoubles;
#pragma unroll
    for (int k = 0; k < kRecDoubles; ++k) {
        o[2 * k] = r[k].hi;
        o[2 * k + 1] = r[k].lo;
    }
}

// One pair in double-double: the field record of the triangle (from rec_dd,
// or rebuilt from the exact input doubles when rec_dd is null) and the pair
// evaluated by the same closed form as the FP64 kernels, its edge loop
// starting at vertex rot (see near_edges).
template <int DEG, int ORDER>
__device__ __noinline__ void pair_dd(const KArgsDD &K, double x, double y, double invh, const double *__restrict__ tri,
                                     const double *__restrict__ nodal, const double *__restrict__ rec_dd, int64_t T,
                                     int64_t t, int rot, double &oI, double &oX, double &oY) {
    dd r[kRecDoubles];
    if (rec_dd) {
        const double *o = rec_dd + t * 2 * kRecDoubles;
#pragma unroll
        for (int k = 0; k < kRecDoubles; ++k) r[k] = dd(o[2 * k], o[2 * k + 1]);
    } else {
        record_dd<ORDER>(invh, tri, nodal, T, t, r);
    }
    dd I, X, Y;
    pair_fwd_rot<DEG, ORDER, dd, DDMath, 1>(K, DDMath(), 0.0, dd(x), dd(y), invh, r, rot, I, X, Y);
    oI = (double)I;
    oX = (double)X;
    oY = (double)Y;
}

// One wavefront owns a window of `groups` x 64 consecutive particles (at most
// kRefGroups; the launch sizes the windows so that the grid has about four
// waves per compute unit, and the waves stride over the windows).  It sweeps the
// window's pairs 64 at a time, one pair per lane, and appends the pairs to
// refine (every pair with a valid triangle in the all-pairs mode, else those
// whose gate fires) to a list in LDS, in pair order; whenever the list is
// full, and at the end of the window, the list is evaluated one pair per lane
// and the results are added to the window's per-particle sums in LDS in list
// order.  The lanes therefore run the costly double-double pairs densely,
// whatever the pairs' distribution over the particles: with a few refined
// pairs per particle group, a whole window makes one evaluation round, whose
// length is that of one double-double pair.  As in the sorted FP64 kernel, a
// list is evaluated in the order of its pairs' near-edge counts, most first,
// each triangle's edge loop starting at its near edges, so that the lanes of
// a round take the same branches.  The sums stay in pair order
// (deterministic).
constexpr int kRefList = 128;
constexpr int kRefGroups = 8;
constexpr int kRefWindow = 64 * kRefGroups;

template <int DEG, int ORDER>
__global__ __launch_bounds__(64) void refine_kernel(const KArgsDD K, RefineGate gate, bool all, int groups, double invh,
                                                     int64_t N, const double *__restrict__ px,
                                                     const double *__restrict__ py, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                     const double *__restrict__ tri,
                                                     const double *__restrict__ nodal, double *__restrict__ I,
                                                     double *__restrict__ Gx, double *__restrict__ Gy,
                                                     double *__restrict__ per_pair, uint8_t *__restrict__ status,
                                                     const double *__restrict__ rec_dd_in,
                                                     unsigned long long dense_min) {
    __shared__ int64_t s_q[kRefList];
    __shared__ uint16_t s_own[kRefList];              // particle within the window
    __shared__ uint8_t s_key[kRefList];               // near-edge count << 2 | rotation
    __shared__ uint8_t s_perm[kRefList];              // evaluation order
    __shared__ double s_res[kRefList][3];
    __shared__ double s_acc[kRefWindow][3];
    __shared__ uint8_t s_any[kRefWindow];
    if (!all && *gate.count == 0) return;       // the forward pass left out no pair
    // the records prepare_dd_kernel built (the same test), else built per pair
    const double *rec_dd = (all || *gate.count >= dense_min) ? rec_dd_in : nullptr;
    const int lane = threadIdx.x;
    const double Rout = K.R[K.npieces - 1], R2 = Rout * Rout;
    const int64_t window = 64 * (int64_t)groups;
    for (int64_t w0 = (int64_t)blockIdx.x * window; w0 < N; w0 += (int64_t)gridDim.x * window) {
        for (int k = lane; k < window; k += 64) {
            s_acc[k][0] = s_acc[k][1] = s_acc[k][2] = 0.0;
            s_any[k] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int n_list = 0;
        // evaluates the listed pairs and adds them to their particles' sums
        auto flush = [&]() {
            // counting sort of the list by near-edge count, most first
            {
                int cnt[4] = {0, 0, 0, 0}, start[4];
                for (int c0 = 0; c0 < n_list; c0 += 64) {
                    const int j = c0 + lane;
                    const int nr = j < n_list ? s_key[j] >> 2 : -1;
#pragma unroll
                    for (int b = 0; b < 4; ++b) cnt[b] += __popcll(__ballot(nr == b));
                }
                start[3] = 0;
                start[2] = cnt[3];
                start[1] = start[2] + cnt[2];
                start[0] = start[1] + cnt[1];
                for (int c0 = 0; c0 < n_list; c0 += 64) {
                    const int j = c0 + lane;
                    const int nr = j < n_list ? s_key[j] >> 2 : -1;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint64_t m = __ballot(nr == b);
                        if (nr == b) s_perm[start[b] + __popcll(m & ((1ull << lane) - 1))] = (uint8_t)j;
                        start[b] += __popcll(m);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int i = lane; i < n_list; i += 64) {
                const int j = s_perm[i];
                const int64_t q = s_q[j];
                const int64_t ip = w0 + s_own[j];
                double vI, vX, vY;
                pair_dd<DEG, ORDER>(K, px[ip], py[ip], invh, tri, nodal, rec_dd, T, tri_idx[q], s_key[j] & 3, vI, vX,
                                    vY);
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
            // lane l adds the entries of the particles l, l + 64, ... in list order
            for (int j = 0; j < n_list; ++j) {
                const int own = s_own[j];
                if ((own & 63) == lane) {
                    s_acc[own][0] += s_res[j][0];
                    s_acc[own][1] += s_res[j][1];
                    s_acc[own][2] += s_res[j][2];
                    s_any[own] = 1;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            n_list = 0;
        };
        for (int g = 0; g < groups; ++g) {
            const int64_t p0 = w0 + 64 * g;
            if (p0 >= N) break;
            const int64_t pid = p0 + lane;
            const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
            // the forward kernels' clamping of the CSR range
            const int64_t q_end = min(max(off[plast], (int64_t)0), P);
            const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
            const int64_t q_begin = __shfl(my_off, 0);
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
                int key = 0;
                if (q < q_end) {
                    const int32_t t = tri_idx[q];
                    if (t >= 0 && t < T) {
                        const int64_t ip = p0 + lo;
                        double ax[3], ay[3];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            ax[k] = (tri[(2 * k) * T + t] - px[ip]) * invh;
                            ay[k] = (tri[(2 * k + 1) * T + t] - py[ip]) * invh;
                        }
                        take = all || gate.fires(ax, ay);
                        if (take) {
                            int rot = 0;
                            const int nr = near_edges(ax, ay, R2, rot);
                            key = nr << 2 | rot;
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
                    s_own[slot] = (uint16_t)(64 * g + lo);
                    s_key[slot] = (uint8_t)key;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                n_list += cnt;
            }
        }
        if (n_list) flush();
        for (int k = lane; k < window; k += 64) {
            const int64_t pid = w0 + k;
            if (pid >= N) break;
            if (all) {
                I[pid] = s_acc[k][0];
                Gx[pid] = s_acc[k][1];
                Gy[pid] = s_acc[k][2];
            } else if (s_any[k]) {
                I[pid] += s_acc[k][0];
                Gx[pid] += s_acc[k][1];
                Gy[pid] += s_acc[k][2];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

template <int ORDER>
void launch_refine_order(int deg, const KArgsDD &K, const RefineGate &g, bool all, double invh, int64_t N,
                         const double *px, const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P,
                         int64_t T, const double *tri, const double *nodal, double *I, double *Gx, double *Gy,
                         double *per_pair, hipStream_t s, uint8_t *status, double *rec_dd) {
    // about four waves per compute unit (the kernel runs one wave per SIMD):
    // the windows grow with N up to kRefGroups groups, so that a few refined
    // pairs per group still make dense evaluation rounds, and the grid still
    // fills the chip when every pair is refined
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 256;
    const int64_t n_groups = (N + 63) / 64, target = 4 * (int64_t)n_cu;
    const int groups = (int)std::min<int64_t>(kRefGroups, std::max<int64_t>(1, n_groups / target));
    // (one round of waves: the kernel holds one wave per SIMD, and a launch
    // that finds nothing to refine costs the dispatch of every block)
    const int64_t want = (n_groups + groups - 1) / groups, cap = (int64_t)n_cu * 4;
    const unsigned blocks = (unsigned)(want < cap ? want : cap);
    const unsigned long long dense_min = 64ull * blocks;      // more refined pairs than one list per wave
    if (rec_dd && T > 0)
        hipLaunchKernelGGL((prepare_dd_kernel<ORDER>), dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, g, all,
                           dense_min, invh, T, tri, nodal, rec_dd);
#define SPHBI_REF(DG)                                                                                          \
    hipLaunchKernelGGL((refine_kernel<DG, ORDER>), dim3(blocks), dim3(64), 0, s, K, g, all, groups, invh, N, px, py, off, \
                       tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, status, rec_dd, dense_min)
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
                  double *per_pair, hipStream_t s, uint8_t *status, double *rec_dd) {
    if (N == 0) return SPHBI_OK;
    const KArgsDD D = make_kargs_dd(K);
    const double invh = 1.0 / h;
    if (order == 0)
        launch_refine_order<0>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s, status, rec_dd);
    else if (order == 1)
        launch_refine_order<1>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status, rec_dd);
    else
        launch_refine_order<3>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status, rec_dd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("refine launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
