// Internal declarations shared by the device library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sphbi.h"

namespace sphbi {

constexpr int kMaxOrder = 3;    // cubic fields
constexpr int kMaxDeg = 11;     // kernel polynomial degree
constexpr int kMaxGauss = SPHBI_MAX_GAUSS;   // Gauss-Legendre points per direction (quadrature path)

// Device-side kernel description, derived on the host from sphbi_kernel.
// R[p], iR[p]  = piece radius and its inverse (units of h)
// b[p][k]      = kernel coefficients of the piece
// bq[p][m][k]  = b_k / (k + 2 + m)     (value, field degree m)
// kbq[p][m][k] = k b_k / (k + 1 + m)   (gradient, field degree m)
// sv[p][m]     = sum_k b_k R^{k+2+m} / (k+2+m)   (value of a unit sector)
// sw[p][m]     = sum_k k b_k R^{k+1+m} / (k+1+m) (gradient of a unit sector)
struct KArgs {
    int npieces;
    int pad;
    double R[2];
    double iR[2];
    double b[2][kMaxDeg + 1];
    double bq[2][kMaxOrder + 1][kMaxDeg + 1];
    double kbq[2][kMaxOrder + 1][kMaxDeg + 1];
    double sv[2][kMaxOrder + 1];
    double sw[2][kMaxOrder + 1];
    double cd;
};

// KArgs whose monomial coefficients b_k are known at compile time to vanish
// in every piece for each bit k of ZM (same layout; the launches pass it in
// place of KArgs).  The Wendland kernels have b_1 = b_3 = ... = 0 below
// their degree (their profile is even to that order), and the instantiations
// for them leave those terms out of the kernel contraction.
template <unsigned ZM>
struct KArgsZ : KArgs {};
template <typename KA>
struct CoefZeros {
    static constexpr unsigned mask = 0;
};
template <unsigned ZM>
struct CoefZeros<KArgsZ<ZM>> {
    static constexpr unsigned mask = ZM;
};
// The zero pattern the instantiations for a degree bound are built for: odd
// k up to the bound's Wendland kernel (C2: b_1; C4: b_1, b_3; C6: b_1, b_3, b_5).
__host__ __device__ constexpr unsigned wendland_zeros(int deg) {
    return deg == 5 ? 0x2u : deg == 8 ? 0xAu : deg == 11 ? 0x2Au : 0u;
}
// Bits k with b_k = 0 in every piece of K.
inline unsigned kernel_zero_mask(const KArgs &K) {
    unsigned m = 0;
    for (int k = 0; k <= kMaxDeg; ++k) {
        bool z = true;
        for (int p = 0; p < K.npieces; ++p) z = z && K.b[p][k] == 0.0;
        if (z) m |= 1u << k;
    }
    return m;
}
// Calls f(KArgsZ<wendland_zeros(DEG)>) when K has that zero pattern, else
// f(K) (the generic instantiation).
template <int DEG, typename F>
inline void with_zero_pattern(const KArgs &K, F &&f) {
    constexpr unsigned wz = wendland_zeros(DEG);
    if constexpr (wz != 0) {
        if ((kernel_zero_mask(K) & wz) == wz) {
            KArgsZ<wz> kz;
            static_cast<KArgs &>(kz) = K;
            f(kz);
            return;
        }
    }
    f(K);
}

// Per-triangle record written by the field preparation kernel: vertices
// (world units) and the field as a polynomial about vertex 0 in units of h,
// A(v0 + h eta) = sum e_ij eta_x^i eta_y^j, ordered e00 e10 e01 e20 e11 e02
// e30 e21 e12 e03.
constexpr int kRecDoubles = 16;

void set_error(const char *fmt, ...);

// A dispatch's grid size in threads is a 32-bit quantity: blocks * threads
// must stay below 2^32.
inline bool grid_fits(int64_t blocks, int threads) {
    return blocks >= 0 && (uint64_t)blocks * (uint64_t)threads < ((uint64_t)1 << 32);
}
// Largest particle and triangle counts of one call: every launch sized by N
// or T uses at most 16 threads per item (plus one block of slack).
constexpr int64_t kMaxItems = ((int64_t)1 << 28) - 256;
// argument checks of sphbi_integrate (everything but the workspace)
int check_integrate_args(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes, int64_t N,
                         const double *px, const double *py, int64_t T, const double *tri, const double *nodal,
                         const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, const double *I,
                         const double *Gx, const double *Gy, const double *per_pair);
KArgs make_kargs(const sphbi_kernel *k, int *deg_out);

// count (nullable): zeroed by the launch (the refinement counter that the
// next forward pass adds to)
int launch_prepare(int order, int64_t T, const double *tri, const double *nodal, double h, double *rec,
                   hipStream_t s, unsigned long long *count = nullptr);
// bytes of the record buffer of T triangles; the refinement counter follows
inline size_t records_bytes(int64_t T) { return (((size_t)(T > 0 ? T : 1) * kRecDoubles * sizeof(double)) + 255) & ~(size_t)255; }
// bytes of the double-double records of the refinement pass (twice the
// doubles of a record), behind the records and the counter
inline size_t dd_records_bytes(int64_t T) { return records_bytes(T) * 2; }
struct RefineGate;
// the whole forward call on prepared-record storage rec: records, FP64 or
// mixed pass, and the double-double refinement the options ask for
int integrate_run(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes, int64_t N,
                  const double *px, const double *py, int64_t T, const double *tri, const double *nodal, double *rec,
                  size_t rec_bytes, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, double *I,
                  double *Gx, double *Gy, double *per_pair, void *stream);
int launch_forward(int order, int deg, int precision, double tau_edge, const KArgs &K, const RefineGate &gate,
                   double h, int64_t N,
                   const double *px, const double *py, const int64_t *offsets, const int32_t *tri_idx,
                   int64_t P, int64_t T, const double *rec, double *I, double *Gx, double *Gy, double *per_pair,
                   hipStream_t s, uint8_t *status = nullptr);

size_t backward_workspace(int64_t T, int64_t P, int n_nodes);
int launch_backward(int order, int deg, int precision, double tau, const KArgs &K, double h, int64_t N,
                    const double *px, const double *py,
                    const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T, const double *tri,
                    const double *nodal, const double *gI, const double *gX, const double *gY, double *dpx,
                    double *dpy, double *dtri, double *dnodal, void *ws, hipStream_t s);
// SPH operators on the boundary (op: SPHBI_OP_*), outputs [N] each; ws of
// operator_workspace(N, T) bytes
size_t operator_workspace(int64_t N, int64_t T);
int launch_operator(int op, int order, int deg, const KArgs &K, double h, int64_t N, const double *px,
                    const double *py, const double *qa, const double *qb, const int64_t *off, const int32_t *tri_idx,
                    int64_t P, int64_t T, const double *tri, const double *fa, const double *fb, double *out_a,
                    double *out_b, void *ws, hipStream_t s);
// boundary pressure with one pressure value per contact; ws as for the operators
int launch_pressure_contact(int deg, const KArgs &K, double h, double rho0, int64_t N, const double *px,
                            const double *py, const double *p_i, const double *rho_i, const int64_t *off,
                            const int32_t *tri_idx, int64_t P, int64_t T, const double *tri, const double *p_pair,
                            double *ax, double *ay, void *ws, hipStream_t s);
// numerical quadrature of the same sums: n_gauss x n_gauss collapsed
// Gauss-Legendre points per triangle (1 <= n_gauss <= kMaxGauss)
int launch_quadrature(int order, int deg, int n_gauss, const KArgs &K, double h, int64_t N, const double *px,
                      const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T,
                      const double *tri, const double *nodal, double *I, double *Gx, double *Gy, hipStream_t s);
// the adjoint pair kernel for linear fields (its own translation unit)
void launch_adjoint_linear(int deg, bool mixed, const KArgs &K, double tau, double invh, int64_t N, const double *px,
                           const double *py, const int64_t *off, const int32_t *tri_idx, int64_t P, int64_t T,
                           const double *tri, const double *nodal, const double *gI, const double *gX,
                           const double *gY, double *dpx, double *dpy, double *pair_grad, hipStream_t s);

}  // namespace sphbi
