/* Driver for the sanitizer build of the CPU oracle (tests/test_sanitizers.py):
 * exercises the definition and closed-form oracles, the pair enumeration and
 * the argument checks on small inputs, including degenerate triangles,
 * particles on edges and vertices and out-of-range indices. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

int oracle_pair(int kid, double h, int nn, double px, double py, const double *tri6, const double *A, double *out);
int oracle_cf_pair(int kid, double h, int nn, double px, double py, const double *tri6, const double *A, double *out);
int oracle_integrate(int kid, double h, int nn, int64_t N, const double *px, const double *py, int64_t T,
                     const double *tri, const double *nodal, const int64_t *off, const int32_t *idx, double *I,
                     double *Gx, double *Gy, double *per_pair, int nthreads);
int64_t oracle_pairlist(int64_t N, const double *px, const double *py, int64_t T, const double *tri, double h,
                        int64_t *offsets, int32_t *tri_idx, int nthreads);

int main(void) {
    const double tris[][6] = {
        {0.0, 0.0, 0.5, 0.1, 0.2, 0.6},        /* particle at a vertex */
        {-0.5, 0.0, 0.5, 0.0, 0.0, 0.7},       /* particle on an edge */
        {-0.5, 0.3, 0.5, 0.3, 0.0, 0.3},       /* zero area */
        {-50, -50, 50, -50, 0, 60},            /* covers the support */
        {1e-9, -0.4, 1e-9, 0.4, 0.8, 0.0},     /* particle 1e-9 from an edge line */
        {0.3, 0.3, 0.3 + 1e-9, 0.3, 0.3, 0.3 + 1e-9},
    };
    const int ntri = (int)(sizeof(tris) / sizeof(tris[0]));
    double A[10];
    for (int k = 0; k < 10; ++k) A[k] = 0.3 + 0.1 * k;
    const int nns[3] = {1, 3, 10};
    double acc = 0.0;
    for (int kid = 0; kid < 4; ++kid)
        for (int a = 0; a < 3; ++a)
            for (int t = 0; t < ntri; ++t) {
                double o[3], c[3];
                if (oracle_pair(kid, 1.0, nns[a], 0.0, 0.0, tris[t], A, o) < 0) return 1;
                if (oracle_cf_pair(kid, 1.0, nns[a], 0.0, 0.0, tris[t], A, c) < 0) return 1;
                acc += o[0] + c[0];
            }
    /* argument checks */
    double o[3];
    if (oracle_pair(9, 1.0, 1, 0.0, 0.0, tris[0], A, o) != -1) return 2;
    if (oracle_pair(0, 0.0, 1, 0.0, 0.0, tris[0], A, o) != -1) return 2;
    if (oracle_pair(0, 1.0, 4, 0.0, 0.0, tris[0], A, o) != -1) return 2;
    /* CSR sums and pair enumeration over a small mesh */
    double tri[6 * 6], nod[10 * 6], px[5], py[5], I[5], Gx[5], Gy[5], pp[3 * 64];
    for (int t = 0; t < ntri; ++t)
        for (int k = 0; k < 6; ++k) tri[k * ntri + t] = tris[t][k];
    for (int k = 0; k < 10 * ntri; ++k) nod[k] = 0.1 * k;
    for (int i = 0; i < 5; ++i) { px[i] = 0.1 * i; py[i] = -0.05 * i; }
    int64_t off[6];
    int32_t idx[64];
    int64_t P = oracle_pairlist(5, px, py, ntri, tri, 0.5, off, NULL, 1);
    if (P < 0 || P > 30) return 3;
    oracle_pairlist(5, px, py, ntri, tri, 0.5, off, idx, 1);
    if (oracle_integrate(1, 0.5, 10, 5, px, py, ntri, tri, nod, off, idx, I, Gx, Gy, pp, 1) < 0) return 4;
    idx[0] = 99;                                /* out-of-range index */
    if (oracle_integrate(1, 0.5, 10, 5, px, py, ntri, tri, nod, off, idx, I, Gx, Gy, NULL, 1) != -2) return 5;
    printf("ok %.6f\n", acc + I[0]);
    return 0;
}
