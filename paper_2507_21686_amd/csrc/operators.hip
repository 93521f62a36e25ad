// SPH operators on the boundary (Sec. 2) and the boundary normal (App. A).
//
// Gradient forms.  The continuous difference and symmetric gradients of a
// field A with density rho (eq. intsphdiffops) are gradient integrals of
// particle-dependent fields.  As the paper prescribes, each pair builds
// pre-weights f_i at the element's nodes, interpolates them with the field's
// own basis and integrates f grad W:
//   difference: f_i = rho_i (A_i - A(x)),                  grad A ~ int f grad W / rho(x),
//   symmetric:  f_i = rho_i (A_i / rho_i^2 + A(x) / rho(x)^2), grad A ~ rho(x) int f grad W.
// The pre-weights are formed before the interpolation, so a large common
// offset of A cancels in A_i - A(x) and not in the integrals.
//
// Divergence and curl of a vector field (A_x, A_y) combine the gradients of
// its components (the equation after eq. improper):
//   div = <grad A_x>_x + <grad A_y>_y,   curl = <grad A_y>_x - <grad A_x>_y.
// Both components go through one closed-form pass (pair_core_n): the
// geometry and the radial terms are shared, only the contraction with each
// component's harmonics is repeated.
//
// Boundary normal (App. A): n(x) = int grad W, the gradient integral of the
// unit field.
//
// Work layout as in the forward kernel: a wavefront owns 64 particles, sweeps
// their pair range one pair per lane and sums per particle with a segmented
// wave scan (deterministic, no atomics).  FP64 throughout.

#include <math.h>

#include "internal.h"
#include "pairmath.h"

namespace sphbi {
namespace {

// op codes shared with the C-ABI
constexpr int kDiff = SPHBI_OP_GRAD_DIFFERENCE, kSym = SPHBI_OP_GRAD_SYMMETRIC, kDivCurl = SPHBI_OP_DIV_CURL,
              kNormal = SPHBI_OP_NORMAL;

__host__ __device__ constexpr int op_edge_unroll(int deg, int order, int nf) {
    return (order >= 2 && deg > 8) || (nf > 1 && order >= 2) ? 1 : 3;
}
// waves per SIMD the register budget is set for: the cubic field's per-pair
// basis (ten nodal polynomials) needs one wave's full budget to stay out of
// scratch memory
__host__ __device__ constexpr int op_waves(int order, int nf) { return order >= 2 ? 1 : (nf > 1 ? 2 : 3); }

// NF = 1: the gradient forms and the normal (op chosen at run time, uniform
// over the grid); NF = 2: divergence and curl.
template <int DEG, int ORDER, int NF>
__global__ __launch_bounds__(256, op_waves(ORDER, NF)) void operator_kernel(const KArgs K, int op, double invh, int64_t N,
                                                       const double *__restrict__ px, const double *__restrict__ py,
                                                       const double *__restrict__ qa, const double *__restrict__ qb,
                                                       const int64_t *__restrict__ off,
                                                       const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                       const double *__restrict__ tri,
                                                       const double *__restrict__ fa, const double *__restrict__ fb,
                                                       double *__restrict__ out_a, double *__restrict__ out_b) {
    constexpr int NN = ORDER == 0 ? 1 : (ORDER == 1 ? 3 : 10);
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
                const double x = px[ip], y = py[ip];
                double v[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
                double ax[3], ay[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ax[i] = (v[2 * i] - x) * invh;
                    ay[i] = (v[2 * i + 1] - y) * invh;
                }
                const double area2 = (ax[1] - ax[0]) * (ay[2] - ay[0]) - (ax[2] - ax[0]) * (ay[1] - ay[0]);
                if (area2 != 0.0) {
                    // nodal values of each field, then the field about the particle
                    double c[10 * NF];
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        double A[10], rec[kRecDoubles];
#pragma unroll
                        for (int k = 0; k < 10; ++k) A[k] = 0.0;
                        if (NF == 2) {
                            const double *src = f == 0 ? fa : fb;
#pragma unroll
                            for (int k = 0; k < NN; ++k) A[k] = src[k * T + t];
                        } else if (op == kNormal) {
                            A[0] = 1.0;
                        } else {
                            const double Ap = qa[ip], rp = qb[ip];
                            const double w = op == kSym ? Ap / (rp * rp) : 0.0;
#pragma unroll
                            for (int k = 0; k < NN; ++k) {
                                const double Ai = fa[k * T + t], ri = fb[k * T + t];
                                A[k] = op == kDiff ? ri * (Ai - Ap) : Ai / ri + ri * w;
                            }
                        }
                        prepare_record<ORDER, double>(v, A, invh, rec);
                        taylor_shift<ORDER, double>(rec + 6, ax[0], ay[0], c + 10 * f);
                    }
                    double oI[NF], oX[NF], oY[NF];
                    pair_core_n<DEG, ORDER, double, ExactMath, op_edge_unroll(DEG, ORDER, NF), NF>(
                        K, ExactMath(), 0.0, ax, ay, area2, c, invh, oI, oX, oY);
                    if (NF == 2) {
                        va = oX[0] + oY[NF - 1];
                        vb = oX[NF - 1] - oY[0];
                    } else {
                        va = oX[0];
                        vb = oY[0];
                    }
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
        double sc = 1.0;
        if (NF == 1 && op == kDiff) sc = 1.0 / qb[pid];
        else if (NF == 1 && op == kSym) sc = qb[pid];
        out_a[pid] = sc * accA;
        out_b[pid] = sc * accB;
    }
}

template <int ORDER, int NF>
void launch_op_deg(int deg, const KArgs &K, int op, double invh, int64_t N, const double *px, const double *py,
                   const double *qa, const double *qb, const int64_t *off, const int32_t *tri_idx, int64_t P,
                   int64_t T, const double *tri, const double *fa, const double *fb, double *out_a, double *out_b,
                   hipStream_t s) {
    const unsigned blocks = (unsigned)(((N + 63) / 64 + 3) / 4);
#define SPHBI_OP(DG)                                                                                              \
    hipLaunchKernelGGL((operator_kernel<DG, ORDER, NF>), dim3(blocks), dim3(256), 0, s, K, op, invh, N, px, py, qa, \
                       qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b)
    if (deg <= 3) SPHBI_OP(3);
    else if (deg <= 5) SPHBI_OP(5);
    else if (deg <= 8) SPHBI_OP(8);
    else SPHBI_OP(11);
#undef SPHBI_OP
}

}  // namespace

int launch_operator(int op, int order, int deg, const KArgs &K, double h, int64_t N, const double *px,
                    const double *py, const double *qa, const double *qb, const int64_t *off, const int32_t *tri_idx,
                    int64_t P, int64_t T, const double *tri, const double *fa, const double *fb, double *out_a,
                    double *out_b, hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    const double invh = 1.0 / h;
    if (op == kNormal) order = 0;
    if (op == kDivCurl) {
        if (order == 0) launch_op_deg<0, 2>(deg, K, op, invh, N, px, py, qa, qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b, s);
        else if (order == 1) launch_op_deg<1, 2>(deg, K, op, invh, N, px, py, qa, qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b, s);
        else launch_op_deg<3, 2>(deg, K, op, invh, N, px, py, qa, qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b, s);
    } else {
        if (order == 0) launch_op_deg<0, 1>(deg, K, op, invh, N, px, py, qa, qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b, s);
        else if (order == 1) launch_op_deg<1, 1>(deg, K, op, invh, N, px, py, qa, qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b, s);
        else launch_op_deg<3, 1>(deg, K, op, invh, N, px, py, qa, qb, off, tri_idx, P, T, tri, fa, fb, out_a, out_b, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("operator launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
