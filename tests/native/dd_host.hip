// Host entry points of the library's double-double arithmetic (ddmath.h),
// built by tests/test_ddmath.py to check it against mpmath.
#include "../../paper_2507_21686_amd/csrc/ddmath.h"

using sphbi::dd;

extern "C" {
void t_log(double h, double l, double *o) { const dd r = sphbi::dd_log(dd(h, l)); o[0] = r.hi; o[1] = r.lo; }
void t_atan2(double yh, double yl, double xh, double xl, double *o) {
    const dd r = sphbi::dd_atan2_q1(dd(yh, yl), dd(xh, xl));
    o[0] = r.hi; o[1] = r.lo;
}
void t_sqrt(double h, double l, double *o) { const dd r = sphbi::dd_sqrt(dd(h, l)); o[0] = r.hi; o[1] = r.lo; }
void t_div(double ah, double al, double bh, double bl, double *o) { const dd r = dd(ah, al) / dd(bh, bl); o[0] = r.hi; o[1] = r.lo; }
void t_mul(double ah, double al, double bh, double bl, double *o) { const dd r = dd(ah, al) * dd(bh, bl); o[0] = r.hi; o[1] = r.lo; }
void t_add(double ah, double al, double bh, double bl, double *o) { const dd r = dd(ah, al) + dd(bh, bl); o[0] = r.hi; o[1] = r.lo; }
void t_fma(double ah, double al, double bh, double bl, double ch, double cl, double *o) { const dd r = fma(dd(ah, al), dd(bh, bl), dd(ch, cl)); o[0] = r.hi; o[1] = r.lo; }
void t_fma1(double a, double bh, double bl, double ch, double cl, double *o) { const dd r = fma(a, dd(bh, bl), dd(ch, cl)); o[0] = r.hi; o[1] = r.lo; }
void t_recip(int n, double *o) { const dd r = sphbi::dd_recip(n); o[0] = r.hi; o[1] = r.lo; }
}
