"""Generates the polynomial coefficients of the FP64 arctangent and logarithm
in fastmath.h (run: python fit_series.py; needs mpmath).

Both are weighted least-squares fits at 50 significant digits on 400
Chebyshev nodes, with the relative error as the weight:
  * atan(u) = u P(u^2) for |u| <= tan(pi/8)   (P of degree 10)
  * log(m)  = s Q(s^2), s = (m - 1)/(m + 1), for m in [1/sqrt 2, sqrt 2]
    (Q approximates 2 atanh(s)/s, degree 8)
The printed maximum relative errors are measured on 2001 points with the
coefficients rounded to double.
"""
import mpmath as mp

mp.mp.dps = 50


def fit(f, smax, deg, npts=400):
    nodes = [smax * (1 - mp.cos(mp.pi * (k + 0.5) / npts)) / 2 for k in range(npts)]
    A = mp.matrix(npts, deg + 1)
    b = mp.matrix(npts, 1)
    for i, s in enumerate(nodes):
        fs = f(s)
        for j in range(deg + 1):
            A[i, j] = s ** j / fs
        b[i] = 1
    c = mp.lu_solve(A.T * A, A.T * b)
    cd = [float(c[j]) for j in range(deg + 1)]
    worst = 0
    for k in range(2001):
        s = smax * mp.mpf(k) / 2000
        p = mp.mpf(0)
        for j in reversed(range(deg + 1)):
            p = p * s + mp.mpf(cd[j])
        worst = max(worst, abs(p / f(s) - 1))
    return cd, float(worst)


def atan_ratio(s):
    return mp.atan(mp.sqrt(s)) / mp.sqrt(s) if s > 0 else mp.mpf(1)


def atanh_ratio(s):
    return 2 * mp.atanh(mp.sqrt(s)) / mp.sqrt(s) if s > 0 else mp.mpf(2)


if __name__ == "__main__":
    t8 = mp.tan(mp.pi / 8)
    c, w = fit(atan_ratio, t8 ** 2, 10)
    print("atan: max rel err", w)
    print(", ".join(repr(x) for x in c))
    r = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    c, w = fit(atanh_ratio, r ** 2, 8)
    print("log: max rel err", w)
    print(", ".join(repr(x) for x in c))
