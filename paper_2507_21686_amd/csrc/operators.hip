// SPH operators on the boundary (Sec. 2) and the boundary normal (App. A).
//
// Gradient forms.  The continuous difference and symmetric gradients of a
// field A with density rho (eq. intsphdiffops) are gradient integrals of
// particle-dependent fields.  The paper forms pre-weights f_i at the
// element's nodes and interpolates them with the field's basis:
//   difference: f_i = rho_i (A_i - A(x)),                      grad A ~ int f grad W / rho(x),
//   symmetric:  f_i = rho_i (A_i / rho_i^2 + A(x) / rho(x)^2),   grad A ~ rho(x) int f grad W.
// The interpolation is linear in the nodal values, so per triangle two
// records are prepared once and every pair combines them in registers
// (forward_pair.h, kFieldComb), f = F1 + (beta_T - gam(x)) F2:
//   difference: F1_i = rho_i (A_i - C_T), F2_i = rho_i, beta_T = C_T, gam = A(x),
//   symmetric:  F1_i = A_i / rho_i,       F2_i = rho_i, beta_T = 0,   gam = -A(x) / rho(x)^2,
// with C_T the mean nodal value of A on the triangle.  Both C_T - A(x) and
// A_i - C_T are differences of nearby values, so a large common offset of A
// cancels there, as it does in the paper's A_i - A(x), and not in the
// integrals.  The pairs then run through the forward pair kernels (sorted by
// near-edge count where that pays), and the per-particle factor is applied
// last.
//
// Divergence and curl of a vector field (A_x, A_y) combine the gradients of
// its components (the equation after eq. improper):
//   div = <grad A_x>_x + <grad A_y>_y,   curl = <grad A_y>_x - <grad A_x>_y.
// Both components go through one closed-form pass (pair_core_n) in the
// sorted forward kernel (kFieldDivCurl): the geometry and the radial terms
// are shared, only the contraction with each component's harmonics is
// repeated.
//
// Boundary normal (App. A): n(x) = int grad W, the forward kernel on records
// of the unit field.
//
// Boundary pressure with one pressure value per contact (App. A, second
// choice): a_i = - sum_q rho0 (p_q / rho0^2 + p_i / rho_i^2) int_T grad W, with
// p_q the pressure at the particle's closest point on the pair's triangle.
// The records hold the constant field -1/rho0 and each pair's result is
// scaled by p_q + rho0^2 p_i / rho_i^2 in the forward kernel
// (kFieldPairWeight).
//
// FP64 throughout; per-particle sums in pair order (deterministic).

#include <math.h>

#include "forward_pair.h"

namespace sphbi {
namespace {

// op codes shared with the C-ABI
constexpr int kDiff = SPHBI_OP_GRAD_DIFFERENCE, kSym = SPHBI_OP_GRAD_SYMMETRIC, kDivCurl = SPHBI_OP_DIV_CURL,
              kNormal = SPHBI_OP_NORMAL;
constexpr int kContact = 100;               // internal: the contact pressure term

// Per-triangle records: rec = vertices and the coefficients of F1 (the
// layout of the forward records), rec2 = the coefficients of F2, then
// beta_T.  F1, F2 per operator as in the header comment; divergence and curl
// take F1 = A_x, F2 = A_y; the normal F1 = 1.
template <int ORDER>
__global__ __launch_bounds__(256) void op_prepare_kernel(int op, int64_t T, const double *__restrict__ tri,
                                                         const double *__restrict__ fa, const double *__restrict__ fb,
                                                         double invh, double unit, double *__restrict__ rec,
                                                         double *__restrict__ rec2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
    double v[6], A[10], B[10];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
#pragma unroll
    for (int k = 0; k < 10; ++k) A[k] = B[k] = 0.0;
    double beta = 0.0;
    if (op == kNormal || op == kContact) {
        A[0] = unit;
    } else {
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            A[k] = fa[k * T + t];
            B[k] = fb[k * T + t];
        }
        if (op == kDiff) {
            double m = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) m += A[k];
            beta = m * (1.0 / NN);
#pragma unroll
            for (int k = 0; k < NN; ++k) A[k] = B[k] * (A[k] - beta);
        } else if (op == kSym) {
#pragma unroll
            for (int k = 0; k < NN; ++k) A[k] = A[k] / B[k];
        }
    }
    double r[kRecDoubles], r2[kRecDoubles];
    prepare_record<ORDER, double>(v, A, invh, r);
    prepare_record<ORDER, double>(v, B, invh, r2);
    double *o = rec + t * kRecDoubles, *o2 = rec2 + t * kRecDoubles;
#pragma unroll
    for (int k = 0; k < kRecDoubles; ++k) o[k] = r[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) o2[k] = r2[6 + k];
    o2[10] = beta;
#pragma unroll
    for (int k = 11; k < kRecDoubles; ++k) o2[k] = 0.0;
}

// gam(x): of the combined field, or the particle's part of the contact
// pressure weight
__global__ void op_gamma_kernel(int op, int64_t N, const double *__restrict__ qa, const double *__restrict__ qb,
                                double rho0, double *__restrict__ gam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    gam[i] = op == kDiff ? qa[i] : (op == kContact ? rho0 * rho0 * qa[i] / (qb[i] * qb[i]) : -qa[i] / (qb[i] * qb[i]));
}

// the per-particle factor of the gradient forms: 1/rho(x) or rho(x)
__global__ void op_scale_kernel(int op, int64_t N, const double *__restrict__ qb, double *__restrict__ a,
                                double *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double sc = op == kDiff ? 1.0 / qb[i] : qb[i];
    a[i] *= sc;
    b[i] *= sc;
}

}  // namespace

size_t operator_workspace(int64_t N, int64_t T) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t Tn = (size_t)(T > 0 ? T : 1), Nn = (size_t)(N > 0 ? N : 1);
    return 2 * al(Tn * kRecDoubles * sizeof(double)) + 2 * al(Nn * sizeof(double));
}

int launch_operator(int op, int order, int deg, const KArgs &K, double h, int64_t N, const double *px,
                    const double *py, const double *qa, const double *qb, const int64_t *off, const int32_t *tri_idx,
                    int64_t P, int64_t T, const double *tri, const double *fa, const double *fb, double *out_a,
                    double *out_b, void *ws, hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t Tn = (size_t)(T > 0 ? T : 1), Nn = (size_t)(N > 0 ? N : 1);
    char *w = (char *)ws;
    double *rec = (double *)w;
    w += al(Tn * kRecDoubles * sizeof(double));
    double *rec2 = (double *)w;
    w += al(Tn * kRecDoubles * sizeof(double));
    double *gam = (double *)w;
    w += al(Nn * sizeof(double));
    double *Ib = (double *)w;
    const double invh = 1.0 / h;
    if (op == kNormal) order = 0;
    if (T > 0) {
        const unsigned tb = (unsigned)((T + 255) / 256);
        if (order == 0) hipLaunchKernelGGL(op_prepare_kernel<0>, dim3(tb), dim3(256), 0, s, op, T, tri, fa, fb, invh, 1.0, rec, rec2);
        else if (order == 1) hipLaunchKernelGGL(op_prepare_kernel<1>, dim3(tb), dim3(256), 0, s, op, T, tri, fa, fb, invh, 1.0, rec, rec2);
        else hipLaunchKernelGGL(op_prepare_kernel<3>, dim3(tb), dim3(256), 0, s, op, T, tri, fa, fb, invh, 1.0, rec, rec2);
    }
    const unsigned nb = (unsigned)((N + 255) / 256);
    if (op == kNormal) {
        int rc = launch_forward(0, deg, SPHBI_FP64, 0.0, K, refine_off(), h, N, px, py, off, tri_idx, P, T, rec, Ib,
                                out_a, out_b, nullptr, s);
        if (rc) return rc;
    } else if (op == kDivCurl) {
        const FwdArgs a{0.0, invh, N, px, py, off, tri_idx, rec, Ib, out_a, out_b, nullptr, P, T, rec2, nullptr};
        if (order == 0) launch_fwd_deg<0, false, kFieldDivCurl>(deg, K, a, s);
        else if (order == 1) launch_fwd_deg<1, false, kFieldDivCurl>(deg, K, a, s);
        else launch_fwd_deg<3, false, kFieldDivCurl>(deg, K, a, s);
    } else {
        hipLaunchKernelGGL(op_gamma_kernel, dim3(nb), dim3(256), 0, s, op, N, qa, qb, 0.0, gam);
        const FwdArgs a{0.0, invh, N, px, py, off, tri_idx, rec, Ib, out_a, out_b, nullptr, P, T, rec2, gam};
        if (order == 0) launch_fwd_deg<0, false, kFieldComb>(deg, K, a, s);
        else if (order == 1) launch_fwd_deg<1, false, kFieldComb>(deg, K, a, s);
        else launch_fwd_deg<3, false, kFieldComb>(deg, K, a, s);
        hipLaunchKernelGGL(op_scale_kernel, dim3(nb), dim3(256), 0, s, op, N, qb, out_a, out_b);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("operator launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi

namespace sphbi {

int launch_pressure_contact(int deg, const KArgs &K, double h, double rho0, int64_t N, const double *px,
                            const double *py, const double *p_i, const double *rho_i, const int64_t *off,
                            const int32_t *tri_idx, int64_t P, int64_t T, const double *tri, const double *p_pair,
                            double *ax, double *ay, void *ws, hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t Tn = (size_t)(T > 0 ? T : 1), Nn = (size_t)(N > 0 ? N : 1);
    char *w = (char *)ws;
    double *rec = (double *)w;
    w += al(Tn * kRecDoubles * sizeof(double));
    double *rec2 = (double *)w;                 // written by the preparation, not read
    w += al(Tn * kRecDoubles * sizeof(double));
    double *gam = (double *)w;
    w += al(Nn * sizeof(double));
    double *Ib = (double *)w;
    const double invh = 1.0 / h;
    if (T > 0)
        hipLaunchKernelGGL(op_prepare_kernel<0>, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, kContact, T, tri,
                           nullptr, nullptr, invh, -1.0 / rho0, rec, rec2);
    hipLaunchKernelGGL(op_gamma_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, kContact, N, p_i, rho_i,
                       rho0, gam);
    const FwdArgs a{0.0, invh, N, px, py, off, tri_idx, rec, Ib, ax, ay, nullptr, P, T, p_pair, gam};
    launch_fwd_deg<0, false, kFieldPairWeight>(deg, K, a, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("pressure launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
