// Forward pair kernel: closed-form int_T A W and int_T A grad W for every
// (particle, triangle) pair, summed per particle.
//
// Decomposition (Sec. 4, eq. intermediateWedge): with the particle at the
// origin of the support-normalised frame (Sec. 2, transform C), a triangle
// with vertices a0, a1, a2 is the signed sum of the three particle-anchored
// triangles (0, a_e, a_{e+1}), each weighted by the sign of its area.  In
// the frame of an edge (x' along the unit normal n towards the edge line at
// distance p, y' along the edge) that triangle is
//     { psi in [psi_a, psi_b], 0 <= r <= min(R, p / cos psi) },
// i.e. the difference of two right-angled stubs anchored at the foot of the
// perpendicular, Q(y_b) - Q(y_a), where each stub is a sector beyond the
// circle crossing and a triangle inside it (Sec. 4.3).  Rotating the field
// into the edge frame is the improper-rotation rule (eq. improper) applied to
// every harmonic at once.
//
// Closed forms (Sec. 5).  For the triangle part of a stub the substitution
// r = p / cos psi turns every moment into radial integrals with Chebyshev
// angular factors (Sec. 5.1):
//     int_0^u cos(n psi) (p/cos psi)^{K+1} dpsi/(K+1)
//         = p/(K+1) sum_j T_n[j] p^j  H_{K-j},
//     int_0^u sin(n psi) (p/cos psi)^{K+1} dpsi/(K+1)
//         = p/(K+1) sum_j U_{n-1}[j] p^j  P_{K-1-j},
// with the hypergeometric radial term H_c = int_p^rho r^c (r^2-p^2)^{-1/2} dr
// (a 2F1 of argument (p/r)^2) evaluated by the contiguous relation
// c H_c = rho^{c-1} y + (c-1) p^2 H_{c-2} from H_0 = asinh(y/p), H_1 = y --
// every term is positive, so the recurrence is stable -- and the powers
// P_e = int_p^rho r^e dr.  The sector parts are the cone formulas of
// Sec. 5.2.  The kernel (Sec. 2, k = sum b_k q^k) and the field harmonics
// (Sec. 3, Table 1 with the gradient of eq. basicdiff) are contracted with
// these radial terms per edge.
//
// Work layout: a wavefront owns 64 consecutive particles; its lanes sweep the
// particles' CSR pair range 64 pairs at a time (one pair per lane), and a
// segmented wave scan (pairs of a particle are contiguous) sums each
// particle's pairs in a fixed order, so the result is deterministic without
// atomics.
//
// Precision: the FP64 instantiation evaluates everything in double; the mixed
// one takes the square roots and reciprocals (and, for P0/P1 fields, the
// sector arctangents) from the FP32 hardware units (precision.h) and keeps
// the logarithm of the radial term, the radial recurrences, the kernel
// contraction and the per-particle sums in FP64.
//
// Field modes (FM), for the SPH operators:
//   kFieldPlain   the record's field: (I, Gx, Gy);
//   kFieldComb    the record's field plus (beta_T - gam[particle]) times a
//                 second field of the same triangle (rec2: its ten
//                 coefficients, then beta_T), formed in the pair's registers
//                 before the evaluation: (I, Gx, Gy) of the combination;
//   kFieldDivCurl the record's field as A_x and rec2's as A_y, both through
//                 one closed-form pass: (0, div, curl);
//   kFieldPairWeight the record's field, each pair's result times
//                 rec2[q] + gam[particle] (rec2 is then one value per pair).
//
// This header is included by forward.hip (plain fields) and operators.hip
// (the other modes); the anonymous namespace keeps each unit's
// instantiations its own.

#pragma once

#include <math.h>

#include <type_traits>

#include "internal.h"
#include "pairmath.h"
#include "refine.h"

namespace sphbi {
namespace {

constexpr int kFieldPlain = 0, kFieldComb = 1, kFieldDivCurl = 2, kFieldPairWeight = 3;

// The pair's record with the combined field: coefficients e + s e2,
// s = rec2[10] - g.
template <int ORDER>
__device__ inline void combine_record(const double *__restrict__ r, const double *__restrict__ r2, double g,
                                      double *rc) {
    constexpr int NC = (ORDER + 1) * (ORDER + 2) / 2;
    const double s = r2[10] - g;
#pragma unroll
    for (int k = 0; k < 6; ++k) rc[k] = r[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) rc[6 + k] = k < NC ? fma(s, r2[k], r[6 + k]) : 0.0;
}

// Waves per SIMD that each instantiation is compiled for (the register
// budget is 512 / waves).  A single wavefront issues an FP64 operation only
// every 5-7 cycles even with independent work (measured on gfx950), so more
// resident waves raise the issue rate as long as the register cut costs
// little spilling.  The table is the fastest of 1-5 waves per instantiation
// on the covering workload (cubic fields 2, linear 3 but 4 for the degree-3
// kernel, constant 4 but 3 for the degree-11 kernel); the cubic-field
// degree-11 variant keeps its edge loop rolled to fit two waves.
__host__ __device__ constexpr int fwd_waves(int deg, int order, bool) {
    return order >= 2 ? 2 : order == 1 ? (deg <= 3 ? 4 : 3) : (deg <= 8 ? 4 : 3);
}
__host__ __device__ constexpr int fwd_edge_unroll(int deg, int order) { return order >= 2 && deg > 8 ? 1 : 3; }

// Divergence and curl of one pair, the vertices taken from rot on (see
// pair_fwd_rot): A_x from the record r, A_y from the coefficients r2, both
// through one closed-form pass (pair_core_n).  Compiled for two waves per
// SIMD with the cubic edge loop rolled: for cubic fields the two fields'
// harmonics then spill about 120 B per lane, and that still runs a quarter
// faster than one wave without spills (0.77 vs 1.04 ms on the covering mesh).
__host__ __device__ constexpr int dc_waves(int) { return 2; }
template <int DEG, int ORDER, typename KA>
__device__ inline void pair_div_curl_rot(const KA &K, double x, double y, double invh, const double *__restrict__ r,
                                         const double *__restrict__ r2, int rot, double &div, double &curl) {
    div = curl = 0.0;
    double ax[3], ay[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ax[i] = (r[2 * i] - x) * invh;
        ay[i] = (r[2 * i + 1] - y) * invh;
    }
    const double area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
    if (area2 == 0.0) return;
    double c[20];
    taylor_shift<ORDER, double>(r + 6, ax[0], ay[0], c);
    taylor_shift<ORDER, double>(r2, ax[0], ay[0], c + 10);
    double bx[3], by[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j1 = i == 2 ? 0 : i + 1, j2 = i == 0 ? 2 : i - 1;
        bx[i] = rot == 0 ? ax[i] : (rot == 1 ? ax[j1] : ax[j2]);
        by[i] = rot == 0 ? ay[i] : (rot == 1 ? ay[j1] : ay[j2]);
    }
    double oI[2], oX[2], oY[2];
    pair_core_n<DEG, ORDER, double, ExactMath, ORDER >= 2 ? 1 : 3, 2>(K, ExactMath(), 0.0, bx, by, area2, c, invh, oI,
                                                                      oX, oY);
    div = oX[0] + oY[1];
    curl = oX[1] - oY[0];
}

template <int DEG, int ORDER, bool MIXED, int FM, typename KA>
__global__ __launch_bounds__(64, fwd_waves(DEG, ORDER, MIXED)) void forward_kernel(const KA K, double tau, double invh, int64_t N,
                                                      const double *__restrict__ px,
                                                      const double *__restrict__ py,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ tri_idx,
                                                      const double *__restrict__ rec, double *__restrict__ I,
                                                      double *__restrict__ Gx, double *__restrict__ Gy,
                                                      double *__restrict__ per_pair, int64_t P, int64_t T,
                                                      const double *__restrict__ rec2,
                                                      const double *__restrict__ gam, const RefineGate gate,
                                                      uint8_t *__restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int64_t p0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
    if (p0 >= N) return;                               // whole wavefront
    const int64_t pid = p0 + lane;
    const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
    // offsets are clamped to [0, P] so that malformed input cannot read past tri_idx
    const int64_t q_end = min(max(off[plast], (int64_t)0), P);
    const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
    const int64_t my_end = pid < N ? min(max(off[pid + 1], my_off), q_end) : q_end;
    const int64_t q_begin = __shfl(my_off, 0);
    double accI = 0.0, accX = 0.0, accY = 0.0;
    unsigned long long n_skip = 0;                     // pairs left to the refinement pass (wave-uniform)
    for (int64_t base = q_begin; base < q_end; base += 64) {
        const int64_t q = base + lane;
        const int64_t qq = q < q_end ? q : q_end - 1;
        // owner lane: largest l with my_off(l) <= qq (uniform 6-step search)
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
            if (lo + step < 64 && om <= qq) lo += step;
        }
        const int owner = lo;
        const int64_t ip = p0 + owner < N ? p0 + owner : N - 1;
        double vI = 0.0, vX = 0.0, vY = 0.0;
        if (q < q_end) {
            const int32_t t = tri_idx[q];
            bool skip = false;      // a pair the refinement pass evaluates in double-double
            if (FM == kFieldPlain && ORDER >= 1 && gate.order && t >= 0 && t < T) {
                const double *r = rec + (int64_t)t * kRecDoubles;
                double gx[3], gy[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gx[k] = (r[2 * k] - px[ip]) * invh;
                    gy[k] = (r[2 * k + 1] - py[ip]) * invh;
                }
                skip = gate.fires(gx, gy);
            }
            if (FM == kFieldPlain && ORDER >= 1 && gate.order) n_skip += __popcll(__ballot(skip));
            if (t >= 0 && t < T && !skip) {   // out-of-range triangle indices contribute nothing
                const double *r = rec + (int64_t)t * kRecDoubles;
                constexpr int EU = fwd_edge_unroll(DEG, ORDER);
                [[maybe_unused]] double rc[FM == kFieldComb ? kRecDoubles : 1];
                if constexpr (FM == kFieldComb) {
                    combine_record<ORDER>(r, rec2 + (int64_t)t * kRecDoubles, gam[ip], rc);
                    r = rc;
                }
                if (MIXED)
                    pair_fwd<DEG, ORDER, double, MixedMath, EU>(K, MixedMath{false, ORDER >= 2}, tau, px[ip], py[ip],
                                                                invh, r, vI, vX, vY);
                else pair_fwd<DEG, ORDER, double, ExactMath, EU>(K, ExactMath(), 0.0, px[ip], py[ip], invh, r, vI, vX,
                                                                 vY);
            }
            if (per_pair && !skip) {
                per_pair[q] = vI;
                per_pair[P + q] = vX;
                per_pair[2 * P + q] = vY;
            }
            if (status) status[q] = !(isfinite(vI) && isfinite(vX) && isfinite(vY));
        }
        // segmented inclusive scan over lanes (segments = owners, contiguous)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double uI = __shfl_up(vI, d), uX = __shfl_up(vX, d), uY = __shfl_up(vY, d);
            const int uo = __shfl_up(owner, d);
            if (lane >= d && uo == owner) {
                vI += uI;
                vX += uX;
                vY += uY;
            }
        }
        // particle lane picks its segment's last lane in this round
        const int64_t s0 = my_off > base ? my_off : base;
        const int64_t s1 = my_end < base + 64 ? my_end : base + 64;
        const int src = s1 > s0 ? (int)(s1 - 1 - base) : 0;
        const double rI = __shfl(vI, src), rX = __shfl(vX, src), rY = __shfl(vY, src);
        if (s1 > s0) {
            accI += rI;
            accX += rX;
            accY += rY;
        }
    }
    if (pid < N) {
        I[pid] = accI;
        Gx[pid] = accX;
        Gy[pid] = accY;
    }
    // one addition per wave: an atomic per 64 pairs on the single counter
    // held the waves up behind it (68% longer on Wendland C4 with cubic
    // fields, where about one pair in twenty is refined)
    if (FM == kFieldPlain && ORDER >= 1 && lane == 0 && n_skip) atomicAdd(gate.count, n_skip);
}

// Sorted variant.  The lanes of a wavefront evaluate different pairs, and an
// edge whose line misses the support circle skips the triangle part (radial
// terms and contraction, the costliest part); lanes that skip it idle while
// the others run it.  Here a wavefront first classifies the pairs of a window
// of its pair range by the number of such near edges (0-3), sorts them by that
// count (counting sort in LDS) and rotates each triangle so that its near
// edges come first; each 64-pair step then runs the triangle part for roughly
// the same edge slots in every lane.  Results go to LDS by pair and every
// particle sums its own pairs in pair order, so the result does not depend on
// the sort and stays deterministic.
//
// One wavefront per block: the waves own different amounts of work, and with
// four per block the block's LDS and slots stay held until its slowest wave
// ends.  With one, every finished wave frees its slot at once (10-15% faster
// on the covering mesh, same results bit for bit).
template <int DEG, int ORDER, bool MIXED, int SW, int FM, typename KA>
__global__ __launch_bounds__(64, FM == kFieldDivCurl ? dc_waves(ORDER) : fwd_waves(DEG, ORDER, MIXED)) void forward_sorted_kernel(
    const KA K, double tau, double invh, int64_t N, const double *__restrict__ px, const double *__restrict__ py,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tri_idx, const double *__restrict__ rec,
    double *__restrict__ I, double *__restrict__ Gx, double *__restrict__ Gy, double *__restrict__ per_pair, int64_t P,
    int64_t T, const double *__restrict__ rec2, const double *__restrict__ gam, const RefineGate gate,
    uint8_t *__restrict__ status) {
    __shared__ double s_res[SW][3];
    __shared__ uint16_t s_perm[SW];
    __shared__ uint8_t s_own[SW];
    __shared__ uint8_t s_key[SW];
    const int lane = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    if (p0 >= N) return;                               // whole wavefront
    const int64_t pid = p0 + lane;
    const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
    const int64_t q_end = min(max(off[plast], (int64_t)0), P);
    const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
    const int64_t my_end = pid < N ? min(max(off[pid + 1], my_off), q_end) : q_end;
    const int64_t q_begin = __shfl(my_off, 0);
    const double Rout = K.R[K.npieces - 1], R2 = Rout * Rout;
    constexpr int EU = fwd_edge_unroll(DEG, ORDER);
    double accI = 0.0, accX = 0.0, accY = 0.0;
    unsigned long long n_skip = 0;                     // pairs left to the refinement pass (wave-uniform)
    for (int64_t sbase = q_begin; sbase < q_end; sbase += SW) {
        const int n = (int)min((int64_t)SW, q_end - sbase);
        // ---- classify: owner lane, number of near edges, rotation
        uint64_t cnt = 0;                              // this lane's items per count, 16 bits each
        for (int c0 = 0; c0 < n; c0 += 64) {
            const int i = c0 + lane;
            const int64_t qq = sbase + (i < n ? i : n - 1);
            int lo = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
                if (lo + step < 64 && om <= qq) lo += step;
            }
            if (i < n) {
                int near = 0, rot = 0;
                const int32_t t = tri_idx[sbase + i];
                if (t >= 0 && t < T) {
                    const int64_t ip = p0 + lo < N ? p0 + lo : N - 1;
                    const double *r = rec + (int64_t)t * kRecDoubles;
                    const double x = px[ip], y = py[ip];
                    double ax[3], ay[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        ax[k] = (r[2 * k] - x) * invh;
                        ay[k] = (r[2 * k + 1] - y) * invh;
                    }
                    near = near_edges(ax, ay, R2, rot);
                    // a pair the refinement pass evaluates in double-double:
                    // no work here (key bit 4), sorted with the cheapest
                    if (FM == kFieldPlain && ORDER >= 1 && gate.order && gate.fires(ax, ay)) {
                        near = 0;
                        rot = 16;
                    }
                }
                if (FM == kFieldPlain && ORDER >= 1 && gate.order) n_skip += __popcll(__ballot(rot == 16));
                s_own[i] = (uint8_t)lo;
                s_key[i] = (uint8_t)(near << 2 | rot);
                cnt += (uint64_t)1 << (16 * near);
            }
        }
        // ---- counting sort by near-edge count, most near edges first
        uint64_t inc = cnt;                            // inclusive scan over lanes
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t u = __shfl_up(inc, d);
            if (lane >= d) inc += u;
        }
        const uint64_t tot = __shfl(inc, 63);
        const uint64_t pre = inc - cnt;
        int start[4];
        {
            const int t3 = (int)(tot >> 48 & 0xffff), t2 = (int)(tot >> 32 & 0xffff), t1 = (int)(tot >> 16 & 0xffff);
            start[3] = 0;
            start[2] = t3;
            start[1] = t3 + t2;
            start[0] = t3 + t2 + t1;
        }
        int run[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) run[b] = start[b] + (int)(pre >> (16 * b) & 0xffff);
        for (int i = lane; i < n; i += 64) {
            const int b = (s_key[i] >> 2) & 3;
            int pos = run[0];
#pragma unroll
            for (int bb = 1; bb < 4; ++bb)
                if (b == bb) pos = run[bb];
#pragma unroll
            for (int bb = 0; bb < 4; ++bb)
                if (b == bb) run[bb] = pos + 1;
            s_perm[pos] = (uint16_t)i;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // ---- evaluate in sorted order; results by pair
        for (int c0 = 0; c0 < n; c0 += 64) {
            const int j = c0 + lane;
            if (j < n) {
                const int item = s_perm[j];
                const int64_t q = sbase + item;
                const int own = s_own[item], key = s_key[item];
                const int64_t ip = p0 + own < N ? p0 + own : N - 1;
                double vI = 0.0, vX = 0.0, vY = 0.0;
                const int32_t t = tri_idx[q];
                const bool skip = key & 16;
                if (t >= 0 && t < T && !skip) {
                    const double *r = rec + (int64_t)t * kRecDoubles;
                    if constexpr (FM == kFieldDivCurl) {
                        pair_div_curl_rot<DEG, ORDER>(K, px[ip], py[ip], invh, r, rec2 + (int64_t)t * kRecDoubles,
                                                      key & 3, vX, vY);
                    } else {
                        [[maybe_unused]] double rc[FM == kFieldComb ? kRecDoubles : 1];
                        if constexpr (FM == kFieldComb) {
                            combine_record<ORDER>(r, rec2 + (int64_t)t * kRecDoubles, gam[ip], rc);
                            r = rc;
                        }
                        if (MIXED)
                            pair_fwd_rot<DEG, ORDER, double, MixedMath, EU>(K, MixedMath{false, ORDER >= 2}, tau,
                                                                            px[ip], py[ip], invh, r, key & 3, vI, vX,
                                                                            vY);
                        else pair_fwd_rot<DEG, ORDER, double, ExactMath, EU>(K, ExactMath(), 0.0, px[ip], py[ip], invh,
                                                                             r, key & 3, vI, vX, vY);
                        if constexpr (FM == kFieldPairWeight) {
                            const double m = rec2[q] + gam[ip];
                            vI *= m;
                            vX *= m;
                            vY *= m;
                        }
                    }
                }
                if (per_pair && !skip) {
                    per_pair[q] = vI;
                    per_pair[P + q] = vX;
                    per_pair[2 * P + q] = vY;
                }
                if (status) status[q] = !(isfinite(vI) && isfinite(vX) && isfinite(vY));
                s_res[item][0] = vI;
                s_res[item][1] = vX;
                s_res[item][2] = vY;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // ---- every particle sums its pairs of this window in pair order
        {
            const int64_t lo = my_off > sbase ? my_off : sbase;
            const int64_t hi = my_end < sbase + n ? my_end : sbase + n;
            for (int64_t k = lo; k < hi; ++k) {
                accI += s_res[k - sbase][0];
                accX += s_res[k - sbase][1];
                accY += s_res[k - sbase][2];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (pid < N) {
        I[pid] = accI;
        Gx[pid] = accX;
        Gy[pid] = accY;
    }
    // one addition per wave: an atomic per 64 pairs on the single counter
    // held the waves up behind it (68% longer on Wendland C4 with cubic
    // fields, where about one pair in twenty is refined)
    if (FM == kFieldPlain && ORDER >= 1 && lane == 0 && n_skip) atomicAdd(gate.count, n_skip);
}

// Sorted or plain kernel per instantiation (measured on the covering
// workload): sorting pays wherever the triangle part is costly (cubic fields,
// and the kernels with more radial terms); for the degree-5 kernel with
// constant or linear fields it costs slightly more than it saves.
__host__ __device__ constexpr bool fwd_sorted(int deg, int order) { return order >= 2 || deg != 5; }

struct FwdArgs {
    double tau, invh;
    int64_t N;
    const double *px, *py;
    const int64_t *off;
    const int32_t *tri_idx;
    const double *rec;
    double *I, *Gx, *Gy, *per_pair;
    int64_t P, T;
    const double *rec2, *gam;      // combined fields only
    RefineGate gate;               // plain fields: pairs left to the refinement pass
    uint8_t *status;               // nullable: per pair, 1 when an output is not finite
};

// Both kernels run one wavefront (64 particles) per block.  A kernel with
// the Wendland zero pattern of its degree bound runs the instantiation that
// leaves those terms out.
template <int DEG, int ORDER, bool MIXED, int FM>
void launch_fwd_t(const KArgs &K, const FwdArgs &a, hipStream_t s) {
    const int64_t waves = (a.N + 63) / 64;
    constexpr int SW = ORDER >= 2 ? 512 : 256;     // LDS: 14 or 7 KB per one-wave block
    with_zero_pattern<DEG>(K, [&](const auto &KZ) {
        using KA = std::decay_t<decltype(KZ)>;
        if constexpr (fwd_sorted(DEG, ORDER) || FM == kFieldDivCurl || FM == kFieldPairWeight)
            hipLaunchKernelGGL((forward_sorted_kernel<DEG, ORDER, MIXED, SW, FM, KA>), dim3((unsigned)waves),
                               dim3(64), 0, s, KZ, a.tau, a.invh, a.N, a.px, a.py, a.off, a.tri_idx, a.rec, a.I, a.Gx,
                               a.Gy, a.per_pair, a.P, a.T, a.rec2, a.gam, a.gate, a.status);
        else
            hipLaunchKernelGGL((forward_kernel<DEG, ORDER, MIXED, FM, KA>), dim3((unsigned)waves), dim3(64), 0, s,
                               KZ, a.tau, a.invh, a.N, a.px, a.py, a.off, a.tri_idx, a.rec, a.I, a.Gx, a.Gy, a.per_pair,
                               a.P, a.T, a.rec2, a.gam, a.gate, a.status);
    });
}

template <int ORDER, bool MIXED, int FM = kFieldPlain>
void launch_fwd_deg(int deg, const KArgs &K, const FwdArgs &a, hipStream_t s) {
    if (deg <= 3) launch_fwd_t<3, ORDER, MIXED, FM>(K, a, s);
    else if (deg <= 5) launch_fwd_t<5, ORDER, MIXED, FM>(K, a, s);
    else if (deg <= 8) launch_fwd_t<8, ORDER, MIXED, FM>(K, a, s);
    else launch_fwd_t<11, ORDER, MIXED, FM>(K, a, s);
}

}  // namespace
}  // namespace sphbi
