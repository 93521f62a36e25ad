// Selection of the pairs that the forward integrals evaluate in
// double-double (refine.hip), shared by the FP64 pair kernels, which leave
// those pairs out of their sums, and the refinement kernel, which adds them.
#pragma once

#include <math.h>

#include "internal.h"
#include "pairmath.h"

namespace sphbi {

// Conditioning gate of a pair.  With the particle at the origin and the
// vertices a_i in units of h, kappa = d_max l_max / |2 area| is how far the
// particle-anchored pieces reach beyond the triangle's width (d_max the
// farthest vertex, l_max the longest edge).  The FP64 closed form loses
// about Kf kappa^order in relative accuracy for a field of polynomial order
// `order` (Kf = sum|b_k| / |sum b_k| of the kernel's monomial form); the gate
// fires when Kf kappa^order exceeds a threshold, in the squared form
//     (d_max^2 l_max^2)^order > g2 (2 area)^(2 order),   g2 = (threshold/Kf)^2.
// It never fires for constant fields (order 0) or degenerate triangles.
// Contraction is off inside: the forward kernel and the refinement kernel
// must take exactly the same decision for every pair.
struct RefineGate {
    int order;      // 0: never fires
    int pad;
    double g2;
    // pairs left out by the FP64 pass (added up by the forward kernel; the
    // refinement kernel does nothing when it reads 0)
    unsigned long long *count;
    __device__ bool fires(const double *ax, const double *ay) const {
#pragma clang fp contract(off)
        if (order == 0) return false;
        const double d0 = ax[0] * ax[0] + ay[0] * ay[0];
        const double d1 = ax[1] * ax[1] + ay[1] * ay[1];
        const double d2 = ax[2] * ax[2] + ay[2] * ay[2];
        const double ex0 = ax[1] - ax[0], ey0 = ay[1] - ay[0];
        const double ex1 = ax[2] - ax[1], ey1 = ay[2] - ay[1];
        const double ex2 = ax[0] - ax[2], ey2 = ay[0] - ay[2];
        const double l0 = ex0 * ex0 + ey0 * ey0, l1 = ex1 * ex1 + ey1 * ey1, l2 = ex2 * ex2 + ey2 * ey2;
        const double a2 = ex0 * (ay[2] - ay[0]) - (ax[2] - ax[0]) * ey0;
        const double dm = fmax(fmax(d0, d1), d2), lm = fmax(fmax(l0, l1), l2);
        const double q = dm * lm, aa = a2 * a2;
        if (!(aa > 0.0)) return false;
        double lhs = q, rhs = aa;
        for (int k = 1; k < order; ++k) {
            lhs = lhs * q;
            rhs = rhs * aa;
        }
        return lhs > g2 * rhs;
    }
};

// A gate that never fires.
inline RefineGate refine_off() { return RefineGate{0, 0, 0.0, nullptr}; }

KArgsDD make_kargs_dd(const KArgs &K);

// The refinement pass: all = true writes I, Gx, Gy (and per_pair) from the
// double-double evaluation of every pair; all = false adds the pairs whose
// gate fires to the outputs of a forward pass run with the same gate.
// rec_dd (dd_records_bytes(T) bytes, or null): storage for the triangles'
// double-double records, built once per call instead of once per pair.
// cursor (one counter, or null): the work counter through which the waves
// share out the particle windows; the all-pairs mode clears it itself, the
// gated mode takes it cleared by the forward pass's field preparation (the
// word after gate.count).  Without one each wave takes a fixed share.
int launch_refine(int order, int deg, const KArgs &K, const RefineGate &gate, bool all, double h, int64_t N,
                  const double *px, const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P,
                  int64_t T, const double *tri, const double *nodal, double *I, double *Gx, double *Gy,
                  double *per_pair, hipStream_t s, uint8_t *status = nullptr, double *rec_dd = nullptr,
                  unsigned long long *cursor = nullptr);

}  // namespace sphbi
