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
// (forward_pair.h, COMB), f = F1 + (beta_T - gam(x)) F2:
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
// Both components go through one closed-form pass (pair_core_n): the
// geometry and the radial terms are shared, only the contraction with each
// component's harmonics is repeated.
//
// Boundary normal (App. A): n(x) = int grad W, the forward kernel on records
// of the unit field.
//
// FP64 throughout; per-particle sums in pair order (deterministic).

#include <math.h>

#include "forward_pair.h"

namespace sphbi {
namespace {

// op codes shared with the C-ABI
constexpr int kDiff = SPHBI_OP_GRAD_DIFFERENCE, kSym = SPHBI_OP_GRAD_SYMMETRIC, kDivCurl = SPHBI_OP_DIV_CURL,
              kNormal = SPHBI_OP_NORMAL;

// Per-triangle records: rec = vertices and the coefficients of F1 (the
// layout of the forward records), rec2 = the coefficients of F2, then
// beta_T.  F1, F2 per operator as in the header comment; divergence and curl
// take F1 = A_x, F2 = A_y; the normal F1 = 1.
template <int ORDER>
__global__ __launch_bounds__(256) void op_prepare_kernel(int op, int64_t T, const double *__restrict__ tri,
                                                         const double *__restrict__ fa, const double *__restrict__ fb,
                                                         double invh, double *__restrict__ rec,
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
    if (op == kNormal) {
        A[0] = 1.0;
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

// gam(x) of the combined field
__global__ void op_gamma_kernel(int op, int64_t N, const double *__restrict__ qa, const double *__restrict__ qb,
                                double *__restrict__ gam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    gam[i] = op == kDiff ? qa[i] : -qa[i] / (qb[i] * qb[i]);
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

__host__ __device__ constexpr int op_edge_unroll(int order) { return order >= 2 ? 1 : 3; }
// waves per SIMD the register budget is set for: two fields' harmonics on
// top of the forward kernel's state
__host__ __device__ constexpr int op_waves(int order) { return order >= 2 ? 1 : 2; }

// Divergence and curl: both components per pair in one closed-form pass.
// Work layout of the plain forward kernel: a wavefront owns 64 particles,
// sweeps their pair range one pair per lane and sums per particle with a
// segmented wave scan.
template <int DEG, int ORDER>
__global__ __launch_bounds__(256, op_waves(ORDER)) void div_curl_kernel(
    const KArgs K, double invh, int64_t N, const double *__restrict__ px, const double *__restrict__ py,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
    const double *__restrict__ rec, const double *__restrict__ rec2, double *__restrict__ out_a,
    double *__restrict__ out_b) {
    const int lane = threadIdx.x & 63;
    const int64_t p0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
    if (p0 >= N) return;
    const int64_t pid = p0 + lane;
    const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
    const int64_t q_end = min(max(off[plast], (int64_t)0), P);
    const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
    const int64_t my_end = pid < N ? min(max(off[pid + 1], my_off), q_end) : q_end;
    const int64_t q_begin = __shfl(my_off, 0);
    double accA = 0.0, accB = 0.0;
    for (int64_t base = q_begin; base < q_end; base += 64) {
        const int64_t q = base + lane;
        const int64_t qq = q < q_end ? q : q_end - 1;
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
            if (lo + step < 64 && om <= qq) lo += step;
        }
        const int owner = lo;
        const int64_t ip = p0 + owner < N ? p0 + owner : N - 1;
        double va = 0.0, vb = 0.0;
        if (q < q_end) {
            const int32_t t = tri_idx[q];
            if (t >= 0 && t < T) {
                const double *r = rec + (int64_t)t * kRecDoubles, *r2 = rec2 + (int64_t)t * kRecDoubles;
                const double x = px[ip], y = py[ip];
                double ax[3], ay[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ax[i] = (r[2 * i] - x) * invh;
                    ay[i] = (r[2 * i + 1] - y) * invh;
                }
                const double area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
                if (area2 != 0.0) {
                    double c[20];
                    taylor_shift<ORDER, double>(r + 6, ax[0], ay[0], c);
                    taylor_shift<ORDER, double>(r2, ax[0], ay[0], c + 10);
                    double oI[2], oX[2], oY[2];
                    pair_core_n<DEG, ORDER, double, ExactMath, op_edge_unroll(ORDER), 2>(
                        K, ExactMath(), 0.0, ax, ay, area2, c, invh, oI, oX, oY);
                    va = oX[0] + oY[1];
                    vb = oX[1] - oY[0];
                }
            }
        }
        // segmented inclusive scan over lanes (segments = owners, contiguous)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double ua = __shfl_up(va, d), ub = __shfl_up(vb, d);
            const int uo = __shfl_up(owner, d);
            if (lane >= d && uo == owner) {
                va += ua;
                vb += ub;
            }
        }
        const int64_t s0 = my_off > base ? my_off : base;
        const int64_t s1 = my_end < base + 64 ? my_end : base + 64;
        const int src = s1 > s0 ? (int)(s1 - 1 - base) : 0;
        const double ra = __shfl(va, src), rb = __shfl(vb, src);
        if (s1 > s0) {
            accA += ra;
            accB += rb;
        }
    }
    if (pid < N) {
        out_a[pid] = accA;
        out_b[pid] = accB;
    }
}

template <int ORDER>
void launch_div_curl_deg(int deg, const KArgs &K, double invh, int64_t N, const double *px, const double *py,
                         const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T, const double *rec,
                         const double *rec2, double *out_a, double *out_b, hipStream_t s) {
    const unsigned blocks = (unsigned)(((N + 63) / 64 + 3) / 4);
#define SPHBI_DC(DG)                                                                                              \
    hipLaunchKernelGGL((div_curl_kernel<DG, ORDER>), dim3(blocks), dim3(256), 0, s, K, invh, N, px, py, off, tri_idx, \
                       P, T, rec, rec2, out_a, out_b)
    if (deg <= 3) SPHBI_DC(3);
    else if (deg <= 5) SPHBI_DC(5);
    else if (deg <= 8) SPHBI_DC(8);
    else SPHBI_DC(11);
#undef SPHBI_DC
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
        if (order == 0) hipLaunchKernelGGL(op_prepare_kernel<0>, dim3(tb), dim3(256), 0, s, op, T, tri, fa, fb, invh, rec, rec2);
        else if (order == 1) hipLaunchKernelGGL(op_prepare_kernel<1>, dim3(tb), dim3(256), 0, s, op, T, tri, fa, fb, invh, rec, rec2);
        else hipLaunchKernelGGL(op_prepare_kernel<3>, dim3(tb), dim3(256), 0, s, op, T, tri, fa, fb, invh, rec, rec2);
    }
    const unsigned nb = (unsigned)((N + 255) / 256);
    if (op == kNormal) {
        int rc = launch_forward(0, deg, SPHBI_FP64, 0.0, K, h, N, px, py, off, tri_idx, P, T, rec, Ib, out_a, out_b,
                                nullptr, s);
        if (rc) return rc;
    } else if (op == kDivCurl) {
        if (order == 0) launch_div_curl_deg<0>(deg, K, invh, N, px, py, off, tri_idx, P, T, rec, rec2, out_a, out_b, s);
        else if (order == 1) launch_div_curl_deg<1>(deg, K, invh, N, px, py, off, tri_idx, P, T, rec, rec2, out_a, out_b, s);
        else launch_div_curl_deg<3>(deg, K, invh, N, px, py, off, tri_idx, P, T, rec, rec2, out_a, out_b, s);
    } else {
        hipLaunchKernelGGL(op_gamma_kernel, dim3(nb), dim3(256), 0, s, op, N, qa, qb, gam);
        const FwdArgs a{0.0, invh, N, px, py, off, tri_idx, rec, Ib, out_a, out_b, nullptr, P, T, rec2, gam};
        if (order == 0) launch_fwd_deg<0, false, true>(deg, K, a, s);
        else if (order == 1) launch_fwd_deg<1, false, true>(deg, K, a, s);
        else launch_fwd_deg<3, false, true>(deg, K, a, s);
        hipLaunchKernelGGL(op_scale_kernel, dim3(nb), dim3(256), 0, s, op, N, qb, out_a, out_b);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("operator launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
