"""The library on non-default HIP streams.

Every call is asynchronous on the stream it is given (the binding passes
torch's current stream).  Results on a side stream must equal those on the
default stream bit for bit, and two integrators on two streams running at
the same time must not disturb each other (each owns its workspace).
"""
import numpy as np
import pytest
import torch

import paper_2507_21686_amd as sb
from paper_2507_21686_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def dev(*a):
    return [torch.as_tensor(np.ascontiguousarray(x), device=DEV) for x in a]


def test_side_stream_matches_default_stream():
    say("streams: side stream vs default stream")
    wl = W.covering_workload(n_side=128, nx=16, ny=32, seed=2, kernel=1, field_order=3)
    px, py, tri, nod = dev(wl.px, wl.py, wl.tri, wl.nodal)
    off, idx = sb.pairlist(px, py, tri, wl.h)
    g = [torch.randn(wl.n_particles, dtype=torch.float64, device=DEV) for _ in range(3)]
    ref = sb.integrate(wl.kernel, wl.h, px, py, tri, nod, off, idx, per_pair=True)
    refb = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off, idx, *g)
    refq = sb.integrate_quadrature(wl.kernel, wl.h, px, py, tri, nod, off, idx, 4)
    torch.cuda.synchronize()
    s = torch.cuda.Stream(device=DEV)              # default priority
    with torch.cuda.stream(s):
        off2, idx2 = sb.pairlist(px, py, tri, wl.h)
        got = sb.integrate(wl.kernel, wl.h, px, py, tri, nod, off2, idx2, per_pair=True)
        gotb = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off2, idx2, *g)
        gotq = sb.integrate_quadrature(wl.kernel, wl.h, px, py, tri, nod, off2, idx2, 4)
        out = [torch.empty(wl.n_particles, dtype=torch.float64, device=DEV) for _ in range(3)]
        sb.integrate_noalloc(wl.kernel, wl.h, px, py, tri, nod, off2, idx2, out)
    s.synchronize()
    assert torch.equal(off, off2) and torch.equal(idx, idx2)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    for a, b in zip(refb, gotb):
        assert torch.equal(a, b)
    for a, b in zip(refq, gotq):
        assert torch.equal(a, b)
    for a, b in zip(ref[:3], out):
        assert torch.equal(a, b)


def test_two_streams_at_once():
    say("streams: two integrators on two streams")
    wa = W.covering_workload(n_side=256, nx=32, ny=64, seed=2, kernel=0, field_order=3)
    wb = W.sliver_stress(seed=3, grid=32, kernel=2, field_order=1)
    ta, tb = dev(wa.px, wa.py, wa.tri, wa.nodal), dev(wb.px, wb.py, wb.tri, wb.nodal)
    oa, ia = sb.pairlist(*ta[:3], wa.h)
    ob, ib = sb.pairlist(*tb[:3], wb.h)
    ra = sb.integrate(wa.kernel, wa.h, *ta, oa, ia)
    rb = sb.integrate(wb.kernel, wb.h, *tb, ob, ib)
    torch.cuda.synchronize()
    ia_, ib_ = sb.Integrator(wa.kernel, wa.h, wa.n_nodes), sb.Integrator(wb.kernel, wb.h, wb.n_nodes)
    sa, sb_ = torch.cuda.Stream(device=DEV), torch.cuda.Stream(device=DEV)
    outs = []
    for _ in range(3):
        with torch.cuda.stream(sa):
            xa = ia_(*ta, oa, ia)
        with torch.cuda.stream(sb_):
            xb = ib_(*tb, ob, ib)
        outs.append((xa, xb))
    torch.cuda.synchronize()
    for xa, xb in outs:
        for a, b in zip(ra, xa):
            assert torch.equal(a, b)
        for a, b in zip(rb, xb):
            assert torch.equal(a, b)
