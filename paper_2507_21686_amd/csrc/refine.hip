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

// The pairs to refine (every pair with a valid triangle in the all-pairs mode,
// else those whose gate fires) are spread unevenly over the particles: on a
// covering mesh with Wendland C4 and cubic fields the 256-particle windows hold
// 0 to 150 of them.  Each wavefront therefore takes windows of 64 particles
// (the first by its index, then from a counter `cursor`, zeroed before the
// launch; without one, every gridDim.x-th window from its own index) until none
// is left, sweeps each window's pairs 64 at a time, one pair per lane, and
// appends the pairs to refine to a list in LDS, in pair order.  The list
// carries over from window to window: whenever it holds kRefBatch entries, the
// first kRefBatch are evaluated one pair per lane, so that the costly
// double-double rounds run full, and a wave ends with one partial batch. The
// results are added to per-particle sums in LDS in list order, one accumulator
// slot per window (kRefSlots of them); a window's sums are written out once it
// has been swept and its last listed pair evaluated. When every slot is taken,
// a batch of what is listed frees them.  As in the sorted FP64 kernel, the
// pairs of a batch are evaluated in the order of their near-edge counts, most
// first, each triangle's edge loop starting at its near edges, so that the
// lanes of a round take the same branches (batches of two rounds measured up to
// 10% slower on the covering meshes). The sums stay in pair order, whichever
// wave takes a window and wherever the batches split it (deterministic).  A
// wave's first window is the one of its own index and the counter hands out the
// rest, so that no wave waits on the counter before it starts.
constexpr int kRefBatch = 64;                 // pairs evaluated together (one round)
constexpr int kRefList = kRefBatch + 64;      // < kRefBatch listed + one sweep step of 64
constexpr int kRefSlots = 16;

template <int DEG, int ORDER>
__global__ __launch_bounds__(64) void refine_kernel(const KArgsDD K, RefineGate gate, bool all, double invh,
                                                     int64_t N, const double *__restrict__ px,
                                                     const double *__restrict__ py, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                     const double *__restrict__ tri,
                                                     const double *__restrict__ nodal, double *__restrict__ I,
                                                     double *__restrict__ Gx, double *__restrict__ Gy,
                                                     double *__restrict__ per_pair, uint8_t *__restrict__ status,
                                                     const double *__restrict__ rec_dd_in,
                                                     unsigned long long dense_min,
                                                     unsigned long long *__restrict__ cursor) {
    __shared__ int64_t s_q[kRefList];
    __shared__ uint8_t s_own[kRefList];               // particle within its window
    __shared__ uint8_t s_slot[kRefList];              // accumulator slot of its window
    __shared__ uint8_t s_key[kRefList];               // near-edge count << 2 | rotation
    __shared__ uint8_t s_perm[kRefBatch];             // evaluation order of a batch
    __shared__ double s_res[kRefBatch][3];
    __shared__ double s_acc[kRefSlots][64][3];
    __shared__ uint8_t s_any[kRefSlots][64];
    __shared__ int64_t s_w0[kRefSlots];               // first particle of the slot's window, -1: free
    __shared__ int s_pend[kRefSlots];                 // listed pairs of the slot's window not yet evaluated
    if (!all && *gate.count == 0) return;       // the forward pass left out no pair
    // the records prepare_dd_kernel built (the same test), else built per pair
    const double *rec_dd = (all || *gate.count >= dense_min) ? rec_dd_in : nullptr;
    const int lane = threadIdx.x;
    const double Rout = K.R[K.npieces - 1], R2 = Rout * Rout;
    auto sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    for (int sl = 0; sl < kRefSlots; ++sl) {
        s_acc[sl][lane][0] = s_acc[sl][lane][1] = s_acc[sl][lane][2] = 0.0;
        s_any[sl][lane] = 0;
    }
    if (lane < kRefSlots) {
        s_w0[lane] = -1;
        s_pend[lane] = 0;
    }
    sync();
    int n_list = 0;
    // writes the sums of slot sl's window and frees the slot
    auto retire = [&](int sl) {
        const int64_t pid = s_w0[sl] + lane;
        if (pid < N) {
            if (all) {
                I[pid] = s_acc[sl][lane][0];
                Gx[pid] = s_acc[sl][lane][1];
                Gy[pid] = s_acc[sl][lane][2];
            } else if (s_any[sl][lane]) {
                I[pid] += s_acc[sl][lane][0];
                Gx[pid] += s_acc[sl][lane][1];
                Gy[pid] += s_acc[sl][lane][2];
            }
        }
        s_acc[sl][lane][0] = s_acc[sl][lane][1] = s_acc[sl][lane][2] = 0.0;
        s_any[sl][lane] = 0;
        sync();
        if (lane == 0) s_w0[sl] = -1;
        sync();
    };
    // evaluates the first min(64, n_list) listed pairs, adds them to their
    // particles' sums and retires the slots left without pending pairs,
    // except `open` (the window being swept)
    auto flush = [&](int open) {
        const int m = n_list < kRefBatch ? n_list : kRefBatch;
        // counting sort of the batch by near-edge count, most first
        {
            int start = 0;
#pragma unroll
            for (int b = 3; b >= 0; --b)
                for (int c0 = 0; c0 < m; c0 += 64) {
                    const int j = c0 + lane;
                    const int nr = j < m ? s_key[j] >> 2 : -1;
                    const uint64_t mk = __ballot(nr == b);
                    if (nr == b) s_perm[start + __popcll(mk & ((1ull << lane) - 1))] = (uint8_t)j;
                    start += __popcll(mk);
                }
        }
        sync();
        for (int i = lane; i < m; i += 64) {
            const int j = s_perm[i];
            const int64_t q = s_q[j];
            const int64_t ip = s_w0[s_slot[j]] + s_own[j];
            double vI, vX, vY;
            pair_dd<DEG, ORDER>(K, px[ip], py[ip], invh, tri, nodal, rec_dd, T, tri_idx[q], s_key[j] & 3, vI, vX, vY);
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
        sync();
        // lane l adds the entries of particle l of every window, in list order
        for (int j = 0; j < m; ++j) {
            if (s_own[j] == lane) {
                const int sl = s_slot[j];
                s_acc[sl][lane][0] += s_res[j][0];
                s_acc[sl][lane][1] += s_res[j][1];
                s_acc[sl][lane][2] += s_res[j][2];
                s_any[sl][lane] = 1;
            }
        }
        // pending counts, then the carried-over entries to the front
        for (int c0 = 0; c0 < m; c0 += 64) {
            const int my_slot = c0 + lane < m ? s_slot[c0 + lane] : -1;
            for (int sl = 0; sl < kRefSlots; ++sl) {
                const int c = __popcll(__ballot(my_slot == sl));
                if (lane == 0 && c) s_pend[sl] -= c;
            }
        }
        const int rest = n_list - m;                  // < 64
        int64_t cq = 0;
        uint8_t co = 0, cs = 0, ck = 0;
        if (lane < rest) {
            cq = s_q[m + lane];
            co = s_own[m + lane];
            cs = s_slot[m + lane];
            ck = s_key[m + lane];
        }
        sync();
        if (lane < rest) {
            s_q[lane] = cq;
            s_own[lane] = co;
            s_slot[lane] = cs;
            s_key[lane] = ck;
        }
        n_list = rest;
        sync();
        for (int sl = 0; sl < kRefSlots; ++sl)
            if (sl != open && s_w0[sl] >= 0 && s_pend[sl] == 0) retire(sl);
    };
    for (int64_t it = 0;; ++it) {
        // the next window: the block's own first, then from the counter (or,
        // without one, the block's fixed share)
        unsigned long long wk = (unsigned long long)(it * gridDim.x + blockIdx.x);
        if (cursor && it > 0) {
            if (lane == 0) wk = gridDim.x + atomicAdd(cursor, 1ull);
            wk = __shfl(wk, 0);
        }
        const int64_t w0 = (int64_t)wk * 64;
        if (w0 >= N) break;                            // every wave reaches this
        // a free slot.  Every taken slot has pending pairs (a window is
        // retired as soon as it has none), and fewer than kRefBatch are listed
        // between windows, so one batch evaluates them all and frees every
        // slot.  The loop ends in any case: each pass evaluates listed pairs,
        // and with none listed no slot has pending pairs, so all can retire.
        int sl = -1;
        for (;;) {
            for (int k = 0; k < kRefSlots && sl < 0; ++k)
                if (s_w0[k] < 0) sl = k;
            if (sl >= 0) break;
            if (n_list > 0) {
                flush(-1);
            } else {
                for (int k = 0; k < kRefSlots; ++k)
                    if (s_w0[k] >= 0) retire(k);
            }
        }
        sync();
        if (lane == 0) {
            s_w0[sl] = w0;
            s_pend[sl] = 0;
        }
        sync();
        const int64_t pid = w0 + lane;
        const int64_t plast = w0 + 64 < N ? w0 + 64 : N;
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
                    const int64_t ip = w0 + lo;
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
            if (take) {
                const int slot = n_list + __popcll(mask & ((1ull << lane) - 1));
                s_q[slot] = q;
                s_own[slot] = (uint8_t)lo;
                s_slot[slot] = (uint8_t)sl;
                s_key[slot] = (uint8_t)key;
            }
            if (lane == 0) s_pend[sl] += cnt;
            n_list += cnt;
            sync();
            if (n_list >= kRefBatch) flush(sl);
        }
        // the window is swept: out at once if nothing of it is pending
        if (s_pend[sl] == 0) retire(sl);
    }
    while (n_list > 0) flush(-1);
}

__global__ void clear_cursor(unsigned long long *cursor) {
    if (threadIdx.x == 0) *cursor = 0;
}

template <int ORDER>
void launch_refine_order(int deg, const KArgsDD &K, const RefineGate &g, bool all, double invh, int64_t N,
                         const double *px, const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P,
                         int64_t T, const double *tri, const double *nodal, double *I, double *Gx, double *Gy,
                         double *per_pair, hipStream_t s, uint8_t *status, double *rec_dd,
                         unsigned long long *cursor) {
    // one wave per SIMD (the kernel's registers allow no more), each taking
    // 64-particle windows until none is left; a launch that finds nothing to
    // refine costs the dispatch of every block, so no more than one round
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 256;
    const int64_t n_windows = (N + 63) / 64, cap = (int64_t)n_cu * 4;
    const unsigned blocks = (unsigned)(n_windows < cap ? n_windows : cap);
    const unsigned long long dense_min = 64ull * blocks;      // more refined pairs than one list per wave
    // the gated mode's counter is cleared with the forward pass's (prepare_kernel)
    if (all && cursor) hipLaunchKernelGGL(clear_cursor, dim3(1), dim3(64), 0, s, cursor);
    if (rec_dd && T > 0)
        hipLaunchKernelGGL((prepare_dd_kernel<ORDER>), dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, g, all,
                           dense_min, invh, T, tri, nodal, rec_dd);
#define SPHBI_REF(DG)                                                                                          \
    hipLaunchKernelGGL((refine_kernel<DG, ORDER>), dim3(blocks), dim3(64), 0, s, K, g, all, invh, N, px, py, off,  \
                       tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, status, rec_dd, dense_min, cursor)
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
                  double *per_pair, hipStream_t s, uint8_t *status, double *rec_dd, unsigned long long *cursor) {
    if (N == 0) return SPHBI_OK;
    const KArgsDD D = make_kargs_dd(K);
    const double invh = 1.0 / h;
    if (order == 0)
        launch_refine_order<0>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status, rec_dd, cursor);
    else if (order == 1)
        launch_refine_order<1>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status, rec_dd, cursor);
    else
        launch_refine_order<3>(deg, D, gate, all, invh, N, px, py, off, tri_idx, P, T, tri, nodal, I, Gx, Gy, per_pair, s,
                               status, rec_dd, cursor);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("refine launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
