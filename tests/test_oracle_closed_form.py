"""The paper's closed-form route (oracle/closed_form.c) against the definition.

The closed-form oracle follows the decomposition of Sec. 4 and the closed
forms of Sec. 5; the definition oracle integrates the definition directly.
They share no arithmetic.  Agreement is checked where the closed forms are
well conditioned: the monomial expansion of the kernel costs a factor
sum|b_k|/|sum b_k| (141 for C2 up to 8.7e3 for C6), and on thin triangles the
particle-anchored pieces extrapolate the P1/P3 polynomial far outside the
triangle, so triangles here have bounded aspect ratio.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2507_21686_amd import workloads as W

# cancellation factor of the monomial kernel expansion per kernel id
KFAC = {0: 141.0, 1: 1109.0, 2: 8704.0, 3: 30.0}


def well_shaped(n, seed, max_ar=6.0):
    """Triangles of size 0.3..2.5 support radii with aspect ratio below max_ar."""
    out = []
    rng_seed = seed
    while len(out) < n:
        tri = W.random_pairs(4 * n, rng_seed, scale_range=(0.3, 2.5))
        rng_seed += 1
        v = tri.reshape(3, 2, -1)
        area2 = np.abs((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
        l2 = np.max([np.sum((v[(i + 1) % 3] - v[i]) ** 2, 0) for i in range(3)], 0)
        ok = (l2 / np.maximum(area2, 1e-300)) < max_ar
        out.extend(list(tri[:, ok].T))
    return np.array(out[:n]).T


@pytest.mark.parametrize("a,m,p,r0,r1", [
    (2, 1, 0.3, 0.4, 0.9), (4, 3, 0.5, 0.55, 1.0), (0, 1, 0.2, 0.2, 1.0), (6, 3, 0.7, 0.75, 0.8),
    (-2, 1, 0.1, 0.3, 0.6), (5, -1, 0.3, 0.3, 1.0), (1, 1, 1e-6, 0.5, 1.0), (3, 5, 0.9, 0.95, 1.0),
    (0, -1, 0.01, 0.02, 1.0), (7, 1, 0.05, 0.06, 0.9), (9, 3, 0.2, 0.21, 1.0), (11, -1, 0.6, 0.6, 1.0),
    (14, 4, 0.4, 0.45, 0.99), (15, 1, 0.999, 0.9995, 1.0)])
def test_radial_term_against_mpmath(a, m, p, r0, r1):
    """J(a,m) = int r^a (1-p^2/r^2)^(m/2) dr, checked by mpmath with r = p cosh t."""
    mp.mp.dps = 30
    P = mp.mpf(p)
    f = lambda t: (P * mp.cosh(t)) ** a * mp.tanh(t) ** m * P * mp.sinh(t)
    ref = float(mp.quad(f, [mp.acosh(mp.mpf(r0) / P), mp.acosh(mp.mpf(r1) / P)]))
    v = oracle.lib().oracle_cf_radial(a, m, p, r0, r1)
    assert abs(v - ref) <= 1e-14 * max(1.0, abs(ref))


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
@pytest.mark.parametrize("nn", [1, 3, 10])
def test_closed_form_matches_definition(kid, nn):
    n = 120
    tri = well_shaped(n, 40 + kid)
    A = np.random.default_rng(kid + nn).standard_normal((nn, n))
    worst = 0.0
    for k in range(n):
        a = oracle.pair(kid, 1.0, 0.0, 0.0, tri[:, k], A[:, k])
        b = oracle.pair(kid, 1.0, 0.0, 0.0, tri[:, k], A[:, k], method="cf")
        worst = max(worst, float(np.abs(a - b).max()) / max(1.0, np.abs(A[:, k]).max()))
    # P1/P3 lose more: the pieces of T2/T3 reach 3 support radii away and the
    # field polynomial is extrapolated over them
    field_tol = {1: 2e-15, 3: 2e-14, 10: 4e-12}[nn]
    assert worst < field_tol * KFAC[kid]


@pytest.mark.parametrize("kid", [0, 3])
def test_closed_form_box_tests(kid):
    tri = W.box_mesh_8()
    s = np.zeros(3)
    for k in range(8):
        s += oracle.pair(kid, 1.0, 0, 0, tri[:, k], [1.0], method="cf")
    np.testing.assert_allclose(s, [1, 0, 0], atol=1e-13)
    nodal = W.vertex_positions(tri)[:, 0]
    s = np.zeros(3)
    for k in range(8):
        s += oracle.pair(kid, 1.0, 0, 0, tri[:, k], nodal[:, k], method="cf")
    np.testing.assert_allclose(s, [0, 1, 0], atol=1e-12)


def test_closed_form_every_case_class_p0():
    """0..3 vertices inside, particle inside/outside: P0 agreement to 1e-13."""
    tri = W.random_pairs(600, 11)
    for k in range(tri.shape[1]):
        a = oracle.pair(0, 1.0, 0, 0, tri[:, k], [1.0])
        b = oracle.pair(0, 1.0, 0, 0, tri[:, k], [1.0], method="cf")
        assert np.abs(a - b).max() < 1e-13


def test_operation_counting_build_reproduces_the_closed_form():
    """The instrumented build (opcount.cpp) evaluates exactly the closed-form
    oracle, bit for bit, and counts a positive number of operations of every
    kind for pairs that reach the support; more vertices inside the support
    mean more pieces (the dispatch of Sec. 4.6) and a field of higher order
    more harmonics."""
    from paper_2507_21686_amd import workloads as W
    tri = W.random_pairs(120, 9, spread=1.3, scale_range=(0.2, 2.5))
    for kid, nn in ((0, 10), (1, 3), (3, 1)):
        A = np.random.default_rng(kid).standard_normal((nn, tri.shape[1]))
        counts, cls, out = oracle.opcount_pairs(kid, tri, A)
        ref = oracle.pairs_normalised(kid, tri, A, method="cf")
        assert np.array_equal(out, ref)
        assert np.all(counts[:, :2] > 0) and set(np.unique(cls)) <= {0, 1, 2, 3}
    A1 = np.ones((1, tri.shape[1]))
    A3 = np.random.default_rng(0).standard_normal((10, tri.shape[1]))
    c1, _, _ = oracle.opcount_pairs(0, tri, A1)
    c3, _, _ = oracle.opcount_pairs(0, tri, A3)
    assert c3.sum() > c1.sum()


def test_committed_op_count_file_matches_its_script():
    """bench.py prices its roofline with oracle/op_count_covering_1M_p3_c2.json;
    the file is what oracle/count_ops.py writes (spot check on the first
    particles of its seeded sample)."""
    import json
    import os
    path = os.path.join(os.path.dirname(oracle.__file__), "op_count_covering_1M_p3_c2.json")
    d = json.load(open(path))
    tot = d["per_pair"]
    assert abs(tot["total"] - (tot["add"] + tot["mul"] + tot["div"] + tot["sqrt"] + tot["transcendental"])) < 1e-6 * tot["total"]
    assert sum(v["fraction"] for v in d["by_case"].values()) == pytest.approx(1.0)
    assert d["written_by"] == "oracle/count_ops.py"
