// Adjoint pair kernel for linear fields (P1), with the FP64 constants as
// scalar-register operands (see sconst).

#include "adjoint_pair.h"

namespace sphbi {

void launch_adjoint_linear(int deg, bool mixed, const KArgs &K, double tau, double invh, int64_t N, const double *px,
                           const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T,
                           const double *tri, const double *nodal, const double *gI, const double *gX,
                           const double *gY, double *dpx, double *dpy, double *pair_grad, hipStream_t s) {
    if (mixed)
        launch_adj_deg<1, true>(deg, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy,
                                pair_grad, s);
    else
        launch_adj_deg<1, false>(deg, K, tau, invh, N, px, py, off, tri_idx, P, T, tri, nodal, gI, gX, gY, dpx, dpy,
                                 pair_grad, s);
}

}  // namespace sphbi
