"""The double-double arithmetic of the refinement path against mpmath (host build).

ddmath.h is compiled for the host with hipcc; every operation and elementary
function must be accurate to a few units of 2^-106 relative (the addition
relative to |a| + |b|, being the short form), the constants (pi/2, ln 2 and
the exact reciprocals 1/n) to their last bit.  The device
build is checked by the refinement tests on the GPU (all-double-double
results against the oracle).
"""
import ctypes as C
import os
import subprocess
import tempfile

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "dd_host.hip")


@pytest.fixture(scope="module")
def ddlib():
    tmp = tempfile.mkdtemp(prefix="ddhost_")
    so = os.path.join(tmp, "libddhost.so")
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-o", so, SRC],
                   check=True, capture_output=True)
    L = C.CDLL(so)
    d = C.c_double
    for f in (L.t_log, L.t_sqrt):
        f.argtypes = [d, d, C.c_void_p]
    for f in (L.t_atan2, L.t_div, L.t_mul, L.t_add):
        f.argtypes = [d, d, d, d, C.c_void_p]
    L.t_recip.argtypes = [C.c_int, C.c_void_p]
    L.t_fma.argtypes = [d, d, d, d, d, d, C.c_void_p]
    L.t_fma1.argtypes = [d, d, d, d, d, C.c_void_p]
    return L


def _val(o):
    return mp.mpf(o[0]) + mp.mpf(o[1])


def test_ddmath_against_mpmath(ddlib):
    mp.mp.dps = 50
    out = np.zeros(2)
    P = out.ctypes.data_as(C.c_void_p)
    rng = np.random.default_rng(0)
    worst = {}

    def rec(name, got, ref):
        worst[name] = max(worst.get(name, 0.0), float(abs(got - ref) / abs(ref)))

    for _ in range(400):
        a = float(np.exp(rng.uniform(-30, 30)))
        al = a * 1e-17 * rng.uniform(-1, 1)
        A = mp.mpf(a) + mp.mpf(al)
        b = float(rng.uniform(-3, 3))
        bl = b * 1e-17 * rng.uniform(-1, 1)
        B = mp.mpf(b) + mp.mpf(bl)
        ddlib.t_log(a, al, P); rec("log", _val(out), mp.log(A)) if abs(mp.log(A)) > 1e-3 else None
        ddlib.t_sqrt(a, al, P); rec("sqrt", _val(out), mp.sqrt(A))
        ddlib.t_div(a, al, b, bl, P); rec("div", _val(out), A / B)
        ddlib.t_mul(a, al, b, bl, P); rec("mul", _val(out), A * B)
        ddlib.t_add(a, al, b, bl, P)
        worst["add"] = max(worst.get("add", 0.0), float(abs(_val(out) - (A + B)) / (abs(A) + abs(B))))
        # fused a b + c, the product unnormalised: within the addition's bound of |a b| + |c|
        c = -a * b * float(rng.uniform(0.9, 1.1))
        cl = c * 1e-17 * rng.uniform(-1, 1)
        Cc = mp.mpf(c) + mp.mpf(cl)
        ddlib.t_fma(a, al, b, bl, c, cl, P)
        worst["fma"] = max(worst.get("fma", 0.0), float(abs(_val(out) - (A * B + Cc)) / (abs(A * B) + abs(Cc))))
        ddlib.t_fma1(b, a, al, c, cl, P)
        worst["fma1"] = max(worst.get("fma1", 0.0),
                            float(abs(_val(out) - (mp.mpf(b) * A + Cc)) / (abs(mp.mpf(b) * A) + abs(Cc))))
        # exact cancellation of the high parts: the low parts' sum, to the bound
        ddlib.t_add(a, al, -a, -al * 0.5, P)
        assert abs(_val(out) - (A - mp.mpf(a) - mp.mpf(al * 0.5))) <= mp.mpf(2) ** -103 * (2 * abs(A))
        y, x = float(np.exp(rng.uniform(-20, 5))), float(np.exp(rng.uniform(-5, 5)))
        ddlib.t_atan2(y, 0.0, x, 0.0, P); rec("atan2", _val(out), mp.atan2(y, x))
    # log near 1 in absolute terms
    for x in (1 - 1e-9, 1 + 3e-12, 0.999, 1.001):
        ddlib.t_log(x, 0.0, P)
        assert abs(_val(out) - mp.log(mp.mpf(x))) < mp.mpf(2) ** -104 * abs(mp.log(mp.mpf(x))) + mp.mpf(2) ** -110
    for n in range(1, 64):
        ddlib.t_recip(n, P)
        rec("recip", _val(out), mp.mpf(1) / n)
    for name, e in worst.items():
        assert e < 2.0 ** -103, (name, e)


def test_ddmath_constants_are_correctly_split():
    """pi/2 and ln 2 as written in ddmath.h: hi is the double nearest to the
    constant and hi + lo is within 2^-106 of it."""
    mp.mp.dps = 50
    txt = open(os.path.join(ROOT, "paper_2507_21686_amd", "csrc", "ddmath.h")).read()
    import re
    for name, ref in (("dd_pi2", mp.pi / 2), ("dd_ln2", mp.log(2))):
        m = re.search(name + r"\(\) \{\s*(?:SPHBI_DD_EXACT\s*)?return dd\(([^,]+), ([^)]+)\);", txt)
        hi, lo = float(m.group(1)), float(m.group(2))
        assert hi == float(ref)
        assert abs(mp.mpf(hi) + mp.mpf(lo) - ref) < mp.mpf(2) ** -106 * ref
