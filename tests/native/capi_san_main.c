/* Driver for the sanitizer build of the library's host code
 * (tests/test_sanitizers.py): kernel presets, options, workspace sizes and
 * every argument check that returns before the device is touched. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/sphbi.h"

#define EXPECT(cond) do { if (!(cond)) { fprintf(stderr, "failed: %s (%s)\n", #cond, sphbi_last_error()); return 1; } } while (0)

int main(void) {
    sphbi_kernel k;
    for (int id = 0; id < 4; ++id) EXPECT(sphbi_kernel_preset(id, &k) == SPHBI_OK && k.c_d > 0);
    EXPECT(sphbi_kernel_preset(9, &k) == SPHBI_EINVAL);
    EXPECT(sphbi_kernel_preset(0, NULL) == SPHBI_EINVAL);
    sphbi_opts o;
    sphbi_default_opts(&o);
    EXPECT(o.precision == SPHBI_FP64 && o.refine == SPHBI_REFINE_AUTO && o.pair_status == NULL);
    sphbi_default_opts(NULL);
    EXPECT(sphbi_integrate_workspace(1000) == 3 * 1000 * 128 + 256);   /* records, counter, double-double records */
    double buf[64] = {0};
    double *p = buf;
    sphbi_kernel_preset(0, &k);
    /* h, n_nodes, NULL arrays, precision, refine mode, gate, sizes */
    EXPECT(sphbi_integrate(&k, &o, 0.0, 1, 4, p, p, 2, p, p, (int64_t *)p, (int32_t *)p, 0, p, p, p, NULL, p, 4096, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_integrate(&k, &o, 1.0, 4, 4, p, p, 2, p, p, (int64_t *)p, (int32_t *)p, 0, p, p, p, NULL, p, 4096, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_integrate(&k, &o, 1.0, 1, 4, NULL, p, 2, p, p, (int64_t *)p, (int32_t *)p, 0, p, p, p, NULL, p, 4096, NULL) == SPHBI_EINVAL);
    sphbi_opts bad = o;
    bad.precision = 7;
    EXPECT(sphbi_integrate(&k, &bad, 1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    bad = o;
    bad.refine = 5;
    EXPECT(sphbi_integrate(&k, &bad, 1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    bad = o;
    bad.refine_gate = -1.0;
    EXPECT(sphbi_integrate(&k, &bad, 1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_integrate(&k, &o, 1.0, 1, (int64_t)1 << 28, p, p, 2, p, p, (int64_t *)p, (int32_t *)p, 0, p, p, p, NULL, p, 4096, NULL) == SPHBI_EUNSUPPORTED);
    EXPECT(sphbi_integrate_noalloc(&k, &o, 1.0, 1, 4, p, p, SPHBI_NOALLOC_MAX_TRIANGLES + 1, p, p, (int64_t *)p, (int32_t *)p, 0, p, p, p, NULL, NULL) == SPHBI_EUNSUPPORTED);
    /* the workspace must be large enough */
    EXPECT(sphbi_integrate(&k, &o, 1.0, 1, 4, p, p, 2, p, p, (int64_t *)p, (int32_t *)p, 0, p, p, p, NULL, p, 8, NULL) == SPHBI_ENOWORKSPACE);
    /* N = 0 is a no-op */
    EXPECT(sphbi_integrate(&k, &o, 1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_OK);
    /* kernel descriptions out of range */
    sphbi_kernel k2 = k;
    k2.degree[0] = 12;
    EXPECT(sphbi_integrate(&k2, &o, 1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    k2 = k;
    k2.n_pieces = 3;
    EXPECT(sphbi_integrate(&k2, &o, 1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    /* operators, quadrature, backward: argument checks */
    EXPECT(sphbi_operator(&k, &o, 7, 1.0, 1, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_integrate_quadrature(&k, 1.0, 1, 0, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_integrate_backward(&k, &o, -1.0, 1, 0, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_pressure_contact(&k, &o, 1.0, 0.0, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, 0, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_mlp_workspace(-1) == 0);
    /* pair lists: sizes, h, an unplanned grid */
    sphbi_grid g;
    memset(&g, 0, sizeof(g));
    int64_t np_ = 0;
    EXPECT(sphbi_pairlist_count(-1, p, p, 0, NULL, 1.0, &g, p, 4096, (int64_t *)p, &np_, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_pairlist_recount(1, p, p, 0, NULL, 0.0, &g, p, 4096, (int64_t *)p, &np_, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_pairlist_recount(1, p, p, 0, NULL, 1.0, &g, p, 4096, (int64_t *)p, &np_, NULL) == SPHBI_EINVAL);
    /* the FP64 probe: iteration count and outputs */
    double fl = 0.0;
    EXPECT(sphbi_probe_fp64_fma(0, p, &fl, NULL) == SPHBI_EINVAL);
    EXPECT(sphbi_probe_fp64_fma(16, p, NULL, NULL) == SPHBI_EINVAL);
    printf("ok\n");
    return 0;
}
