// Numerical quadrature of the boundary integrals, for comparison with the
// closed form (the quadrature-convergence evaluation of Sec. 6.2).
//
// The paper compares its analytic integrals against quadrature rules that
// cover the whole triangle: inside the support the integrand A W is smooth,
// but the support circle cuts through triangles it only partly covers, and
// there the compact cut-off limits what a rule can reach (Sec. 6.1).  This
// path evaluates the same sums as sphbi_integrate,
//   I(x) = sum_T int_T A W(|x - x'|) dx',  G(x) = sum_T int_T A grad_x W dx',
// with a collapsed (Duffy) tensor Gauss-Legendre rule of n x n points per
// triangle: barycentric coordinates L1 = u, L2 = (1 - u) v, L0 = 1 - L1 - L2
// for (u, v) in [0, 1]^2, area element |2 area| (1 - u) du dv.  The rule is
// exact for fields times polynomials of total degree <= 2n - 2 in (L1, L2).
//
// The Gauss-Legendre nodes are computed on the host by Newton's iteration on
// the three-term Legendre recurrence and handed to the kernel by value.  Sums
// are taken in a fixed order (deterministic).  FP64.

#include <math.h>

#include "internal.h"

namespace sphbi {
namespace {

// the kernel polynomial only (the closed form's tables are not needed here)
struct QuadKernel {
    int npieces;
    int pad;
    double R[2];
    double b[2][kMaxDeg + 1];
    double cd;
};

struct QuadRule {
    int n;
    int pad;
    double x[kMaxGauss];   // nodes on [0, 1]
    double w[kMaxGauss];   // weights on [0, 1] (sum 1)
};

// k(q) and k'(q) of the piecewise kernel polynomial (pieces add where q < R_p)
__device__ inline void kernel_and_slope(const QuadKernel &K, int deg, double q, double &k, double &dk) {
    k = 0.0;
    dk = 0.0;
    for (int p = 0; p < K.npieces; ++p) {
        if (!(q < K.R[p])) continue;
        double v = K.b[p][deg], d = deg * K.b[p][deg];
        for (int j = deg - 1; j >= 0; --j) {
            v = v * q + K.b[p][j];
            if (j >= 1) d = d * q + j * K.b[p][j];
        }
        k += v;
        dk += d;
    }
}

// field at barycentric (L0, L1, L2): P0 constant, P1 barycentric, P3 cubic
// Lagrange on v0, v1, v2, the edge nodes of v0v1, v1v2, v2v0 at 1/3 and 2/3
// from the first vertex, and the centroid
template <int NN>
__device__ inline double field_at(const double *A, double L0, double L1, double L2) {
    if constexpr (NN == 1) {
        return A[0];
    } else if constexpr (NN == 3) {
        return L0 * A[0] + L1 * A[1] + L2 * A[2];
    } else {
        const double L[3] = {L0, L1, L2};
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) s += 0.5 * L[a] * (3.0 * L[a] - 1.0) * (3.0 * L[a] - 2.0) * A[a];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int a = e, b = (e + 1) % 3;
            const double ab = 4.5 * L[a] * L[b];
            s += ab * (3.0 * L[a] - 1.0) * A[3 + 2 * e];     // 1/3 from a: L_a = 2/3
            s += ab * (3.0 * L[b] - 1.0) * A[4 + 2 * e];     // 2/3 from a: L_b = 2/3
        }
        s += 27.0 * L0 * L1 * L2 * A[9];
        return s;
    }
}

// Thread layout: every particle gets n threads; thread a of a particle takes
// the outer Gauss row a (n points) of each of its pairs, in pair order, and
// the n row sums are added in row order through LDS.  A block of 256 threads
// holds ppb = floor(256 / n) particles.  n threads per particle keep the chip
// busy when there are few particles; the sums stay deterministic, and a pair
// with an invalid index changes nothing.
template <int NN>
__global__ __launch_bounds__(256) void quadrature_kernel(const QuadKernel K, const QuadRule Q, int deg, double h,
                                                         int ppb, int64_t N, const double *__restrict__ px,
                                                         const double *__restrict__ py,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ tri_idx, int64_t P, int64_t T,
                                                         const double *__restrict__ tri,
                                                         const double *__restrict__ nodal, double *__restrict__ I,
                                                         double *__restrict__ Gx, double *__restrict__ Gy) {
    __shared__ double s_x[kMaxGauss], s_w[kMaxGauss];
    __shared__ double s_red[3][256];
    const int n = Q.n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        s_x[k] = Q.x[k];
        s_w[k] = Q.w[k];
    }
    __syncthreads();
    const int slot = threadIdx.x / n, a = threadIdx.x - slot * n;
    const int64_t i = (int64_t)blockIdx.x * ppb + slot;
    const bool act = slot < ppb && i < N;
    const double invh = 1.0 / h;
    double si = 0.0, sx = 0.0, sy = 0.0;
    if (act) {
        const double x = px[i], y = py[i];
        int64_t lo = off[i], hi = off[i + 1];
        lo = lo < 0 ? 0 : (lo > P ? P : lo);
        hi = hi < lo ? lo : (hi > P ? P : hi);
        const double u = s_x[a], wu = s_w[a] * (1.0 - u);
        for (int64_t q = lo; q < hi; ++q) {
            const int32_t t = tri_idx[q];
            if (t < 0 || t >= T) continue;
            const double ax = tri[t], ay = tri[T + t], bx = tri[2 * T + t], by = tri[3 * T + t];
            const double cx = tri[4 * T + t], cy = tri[5 * T + t];
            double A[NN];
#pragma unroll
            for (int k = 0; k < NN; ++k) A[k] = nodal[k * T + t];
            const double area2 = fabs((bx - ax) * (cy - ay) - (by - ay) * (cx - ax));
            double ri = 0.0, rx = 0.0, ry = 0.0;
            for (int b = 0; b < n; ++b) {
                const double L1 = u, L2 = (1.0 - u) * s_x[b], L0 = 1.0 - L1 - L2;
                const double dx = (x - (L0 * ax + L1 * bx + L2 * cx)) * invh;
                const double dy = (y - (L0 * ay + L1 * by + L2 * cy)) * invh;
                const double r = sqrt(dx * dx + dy * dy);
                double k, dk;
                kernel_and_slope(K, deg, r, k, dk);
                const double fw = field_at<NN>(A, L0, L1, L2) * s_w[b];
                ri += fw * k;
                if (r > 0.0) {
                    const double g = fw * dk / r;
                    rx += g * dx;
                    ry += g * dy;
                }
            }
            const double c = area2 * wu;
            si += c * ri;
            sx += c * rx;
            sy += c * ry;
        }
    }
    s_red[0][threadIdx.x] = si;
    s_red[1][threadIdx.x] = sx;
    s_red[2][threadIdx.x] = sy;
    __syncthreads();
    if (act && a == 0) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int k = 0; k < n; ++k) {             // rows in order; threadIdx.x + k < ppb * n <= 256
            t0 += s_red[0][threadIdx.x + k];
            t1 += s_red[1][threadIdx.x + k];
            t2 += s_red[2][threadIdx.x + k];
        }
        const double sv = K.cd * invh * invh, sg = sv * invh;
        I[i] = sv * t0;
        Gx[i] = sg * t1;
        Gy[i] = sg * t2;
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's iteration on P_n,
// evaluated by the recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}, from
// the usual cosine first guesses; mapped to [0, 1].
void gauss_legendre01(int n, double *x, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double t = cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2 * k + 1) * t * p1 - k * p0) / (k + 1);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);       // P_n'(t), p0 = P_{n-1}
            const double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 1; k < n; ++k) {
            const double p2 = ((2 * k + 1) * t * p1 - k * p0) / (k + 1);
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = 0.5 * (1.0 - t);                          // ascending on [0, 1]
        w[i] = 1.0 / ((1.0 - t * t) * dp * dp);          // 2/((1-t^2) P_n'^2), halved
    }
}

}  // namespace

int launch_quadrature(int order, int deg, int n_gauss, const KArgs &K, double h, int64_t N, const double *px,
                      const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T,
                      const double *tri, const double *nodal, double *I, double *Gx, double *Gy, hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    QuadKernel QK{};
    QK.npieces = K.npieces;
    QK.cd = K.cd;
    for (int p = 0; p < 2; ++p) {
        QK.R[p] = K.R[p];
        for (int k = 0; k <= kMaxDeg; ++k) QK.b[p][k] = K.b[p][k];
    }
    QuadRule Q{};
    Q.n = n_gauss;
    gauss_legendre01(n_gauss, Q.x, Q.w);
    const int ppb = 256 / n_gauss;
    if (!grid_fits((N + ppb - 1) / ppb, 256)) {
        set_error("too many particles for one quadrature launch (%lld; at most %lld at n_gauss = %d)", (long long)N,
                  (long long)((((int64_t)1 << 32) / 256 - 1) * ppb), n_gauss);
        return SPHBI_EUNSUPPORTED;
    }
    const unsigned nb = (unsigned)((N + ppb - 1) / ppb);
    if (order == 0)
        hipLaunchKernelGGL(quadrature_kernel<1>, dim3(nb), dim3(256), 0, s, QK, Q, deg, h, ppb, N, px, py, off, tri_idx, P,
                           T, tri, nodal, I, Gx, Gy);
    else if (order == 1)
        hipLaunchKernelGGL(quadrature_kernel<3>, dim3(nb), dim3(256), 0, s, QK, Q, deg, h, ppb, N, px, py, off, tri_idx, P,
                           T, tri, nodal, I, Gx, Gy);
    else
        hipLaunchKernelGGL(quadrature_kernel<10>, dim3(nb), dim3(256), 0, s, QK, Q, deg, h, ppb, N, px, py, off, tri_idx, P,
                           T, tri, nodal, I, Gx, Gy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("quadrature launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
