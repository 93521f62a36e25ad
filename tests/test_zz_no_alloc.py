"""The allocation-free forward entry point against sphbi_integrate.

sphbi_integrate_noalloc keeps its per-triangle records in a fixed per-GPU
array instead of a workspace.  Its results must equal sphbi_integrate's bit
for bit (the same kernels run on the same records), on two calls in a row,
the second with a smaller input, so that the array's leftovers from the
first call cannot leak into the second.
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


def _dev(*a):
    return [torch.as_tensor(np.ascontiguousarray(x), device=DEV) for x in a]


def _both(wl, precision=sb.FP64):
    px, py, tri, nod = _dev(wl.px, wl.py, wl.tri, wl.nodal)
    off, idx = sb.pairlist(px, py, tri, wl.h)
    ref = sb.integrate(wl.kernel, wl.h, px, py, tri, nod, off, idx, per_pair=True, precision=precision)
    N, P = px.numel(), idx.numel()
    out = [torch.full((N,), np.nan, dtype=torch.float64, device=DEV) for _ in range(3)]
    pp = torch.full((3, P), np.nan, dtype=torch.float64, device=DEV)
    sb.integrate_noalloc(wl.kernel, wl.h, px, py, tri, nod, off, idx, out, per_pair=pp, precision=precision)
    torch.cuda.synchronize()
    for a, b in zip(ref[:3], out):
        assert torch.equal(a, b)
    assert torch.equal(ref[3], pp)
    return P


def test_noalloc_matches_integrate_two_calls_shrinking():
    big = W.covering_workload(n_side=256, nx=64, ny=128, seed=2)          # 16,384 triangles, P3
    small = W.covering_workload(n_side=64, nx=8, ny=16, seed=5, kernel=sb.WENDLAND_C4, field_order=1)
    say(f"noalloc: first call T={big.n_triangles} N={big.n_particles}")
    p1 = _both(big)
    say(f"noalloc: second call T={small.n_triangles} N={small.n_particles}")
    p2 = _both(small)
    assert p1 > p2 > 0


def test_noalloc_mixed_and_band_wall():
    say("noalloc: mixed precision, covering mesh")
    _both(W.covering_workload(n_side=128, nx=16, ny=32, seed=7, kernel=sb.WENDLAND_C6, field_order=3), sb.MIXED)
    say("noalloc: band wall")
    _both(W.band_wall(seed=1))


def test_noalloc_limits_and_empty():
    say("noalloc: limits")
    T = sb.NOALLOC_MAX_TRIANGLES + 1
    px, py = _dev(np.zeros(4), np.zeros(4))
    tri = torch.zeros((6, T), dtype=torch.float64, device=DEV)
    nod = torch.zeros((1, T), dtype=torch.float64, device=DEV)
    off = torch.zeros(5, dtype=torch.int64, device=DEV)
    idx = torch.zeros(0, dtype=torch.int32, device=DEV)
    out = [torch.zeros(4, dtype=torch.float64, device=DEV) for _ in range(3)]
    with pytest.raises(sb.SphbiError, match="EUNSUPPORTED"):
        sb.integrate_noalloc(0, 0.1, px, py, tri, nod, off, idx, out)
    # no pairs: zeros, not leftovers of an earlier call
    out = [torch.full((4,), 7.0, dtype=torch.float64, device=DEV) for _ in range(3)]
    tri = torch.zeros((6, 3), dtype=torch.float64, device=DEV)
    nod = torch.zeros((1, 3), dtype=torch.float64, device=DEV)
    sb.integrate_noalloc(0, 0.1, px, py, tri, nod, off, idx, out)
    torch.cuda.synchronize()
    for o in out:
        assert torch.all(o == 0)


def test_noalloc_graph_replays():
    """The allocation-free call captured in a HIP graph (its intended caller):
    every replay, with new nodal values and positions written in place and
    eager library calls between the replays, equals sphbi_integrate run
    eagerly on the same inputs, bit for bit (Wendland C4 with cubic fields,
    so that the refinement pass runs inside the graph too)."""
    wl = W.covering_workload(n_side=128, nx=16, ny=32, seed=7, kernel=sb.WENDLAND_C4, field_order=3)
    say(f"noalloc graph: T={wl.n_triangles} N={wl.n_particles}")
    px, py, tri, nod = _dev(wl.px, wl.py, wl.tri, wl.nodal)
    off, idx = sb.pairlist(px, py, tri, wl.h)
    N = px.numel()
    out = [torch.zeros(N, dtype=torch.float64, device=DEV) for _ in range(3)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):             # one eager call on the capture stream first
        sb.integrate_noalloc(wl.kernel, wl.h, px, py, tri, nod, off, idx, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sb.integrate_noalloc(wl.kernel, wl.h, px, py, tri, nod, off, idx, out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(21)
    for rep in range(4):
        nod.copy_(torch.as_tensor(rng.standard_normal(wl.nodal.shape), device=DEV))
        px.copy_(torch.as_tensor(wl.px + rng.uniform(-0.1, 0.1, N) * wl.h, device=DEV))
        for o in out:
            o.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = sb.integrate(wl.kernel, wl.h, px, py, tri, nod, off, idx)
        torch.cuda.synchronize()
        for a, b in zip(ref[:3], out):
            assert torch.equal(a, b), rep
    say("  4 replays equal to the eager call")
