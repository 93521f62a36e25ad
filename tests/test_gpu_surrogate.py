"""GPU parity of the learned surrogate's kernels against the CPU reference.

* features: bit-exact (every geometric decision is taken in FP64 without
  fused multiply-adds on both sides);
* network forward and loss gradient: against oracle/mlp.py evaluated with
  the same bfloat16 rounding of weights, layer inputs and backward operands
  (the only differences left are FP32 accumulation order and the rare
  bfloat16 rounding flip it causes);
* Adam: against the reference update in FP64;
* fused serving kernel: against the same reference on the pairs of a mesh;
* router: with every pair flagged the result is the closed form; with none
  flagged it is the network's prediction.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as ref
import paper_2507_21686_amd as sb
from paper_2507_21686_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a), device=DEV)
    return t if dtype is None else t.to(dtype)


def mesh_pairs(n_side=64, seed=2):
    wl = W.covering_workload(n_side=n_side, nx=max(1, 128 * n_side // 1024), ny=max(1, 256 * n_side // 1024),
                             seed=seed, kernel=0, field_order=0)
    px, py, tri = dev(wl.px), dev(wl.py), dev(wl.tri)
    off, idx = sb.pairlist(px, py, tri, wl.h)
    torch.cuda.synchronize()
    return wl, px, py, tri, off, idx


def owners(off):
    off = off.cpu().numpy()
    return np.repeat(np.arange(len(off) - 1), np.diff(off))


def test_features_bit_exact():
    wl, px, py, tri, off, idx = mesh_pairs()
    say(f"features: pairs={idx.numel()}")
    f, r = sb.surrogate_features(px, py, tri, wl.h, off, idx)
    torch.cuda.synchronize()
    own = owners(off)
    t = idx.cpu().numpy()
    rf, rr = ref.features(wl.px[own], wl.py[own], wl.tri[:, t], wl.h)
    np.testing.assert_array_equal(f.cpu().numpy(), rf.astype(np.float32))
    np.testing.assert_array_equal(r.cpu().numpy(), rr.astype(np.float32))
    # edge geometry: particle at a vertex, on an edge, degenerate triangle
    tri2 = np.array([[0.0, 0.0, 0.05, 0.01, 0.02, 0.06], [-0.05, 0.0, 0.05, 0.0, 0.0, 0.07],
                     [-0.05, 0.03, 0.05, 0.03, 0.0, 0.03], [0.1, 0.0, 0.15, 0.0, 0.12, 0.05]]).T.copy()
    n = tri2.shape[1]
    f2, r2 = sb.surrogate_features(dev(np.zeros(n)), dev(np.zeros(n)), dev(tri2), 0.1,
                                   dev(np.arange(n + 1, dtype=np.int64)), dev(np.arange(n, dtype=np.int32)))
    rf2, rr2 = ref.features(np.zeros(n), np.zeros(n), tri2, 0.1)
    np.testing.assert_array_equal(f2.cpu().numpy(), rf2.astype(np.float32))
    np.testing.assert_array_equal(r2.cpu().numpy(), rr2.astype(np.float32))


def close_bf16(got, want, what):
    """The reference applies the same bfloat16 roundings, but the matrix cores
    add in their own order, so a value on a rounding boundary may round the
    other way now and then: one bfloat16 step (2^-8 of that value) in one
    operand, carried through the later layers.  Measured over these tests:
    maxima 4e-8 ... 7.2e-4 of the scale, medians below 3e-8."""
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    scale = np.abs(want).max()
    err = np.abs(got - want) / scale
    say(f"  {what}: max {err.max():.2e} median {np.median(err):.2e} (scale {scale:.3e})")
    assert err.max() < 3e-3 and np.median(err) < 1e-6, what


@pytest.mark.parametrize("B", [1, 77, 1000])
def test_mlp_forward_vs_reference(B):
    say(f"mlp forward B={B}")
    p = ref.init_params(3)
    x = np.random.default_rng(B).standard_normal((B, 8)).astype(np.float32)
    out = sb.mlp_forward(dev(p), dev(x)).cpu().numpy()
    want = ref.forward(p, x, round_bf16=True)
    close_bf16(out, want, "outputs")


def test_mlp_loss_grad_vs_reference():
    B = 777
    rng = np.random.default_rng(11)
    p = (ref.init_params(4) * 1.5).astype(np.float32)
    x = rng.standard_normal((B, 8)).astype(np.float32)
    t = rng.standard_normal((B, 3)).astype(np.float32)
    scale = np.array([0.5, 0.8, 0.8])
    lam = 0.05
    say("mlp loss/grad")
    loss, g = sb.mlp_loss_grad(dev(p), dev(x), dev(t), scale, lam)
    loss, g = float(loss.cpu()), g.cpu().numpy()
    L, gref = ref.loss_and_grad(p, x, t, scale, lam, round_bf16=True)
    say(f"  loss {loss:.6e} ref {L:.6e}")
    assert abs(loss - L) <= 1e-4 * abs(L)
    o = 0
    for li, (i, n) in enumerate(ref.LAYERS):
        for part, size in (("W", i * n), ("b", n)):
            close_bf16(g[o:o + size], gref[o:o + size], f"layer {li + 1} {part}")
            o += size
    # determinism
    _, g2 = sb.mlp_loss_grad(dev(p), dev(x), dev(t), scale, lam)
    assert np.array_equal(g2.cpu().numpy(), g)


def test_adam_vs_reference():
    say("adam")
    rng = np.random.default_rng(2)
    n = 5000
    p = rng.standard_normal(n).astype(np.float32)
    m = (rng.standard_normal(n) * 0.1).astype(np.float32)
    v = rng.uniform(0, 0.1, n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    tp, tm, tv, tg = dev(p), dev(m), dev(v), dev(g)
    sb.adam_step(tp, tm, tv, tg, 1e-3, 7)
    pr, mr, vr = ref.adam(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64), g.astype(np.float64),
                          7, 1e-3)
    np.testing.assert_allclose(tp.cpu().numpy(), pr, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(tm.cpu().numpy(), mr, rtol=2e-6, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), vr, rtol=2e-6, atol=1e-9)


def serve_reference(wl, off, idx, p, mean, std, A):
    """Per-pair values of the serving path from the CPU reference (no routing)."""
    own = owners(off)
    t = idx.cpu().numpy()
    f, rot = ref.features(wl.px[own], wl.py[own], wl.tri[:, t], wl.h)
    y = ref.forward(p, f.astype(np.float32), round_bf16=True)
    y3 = y[:, :3] * std + mean
    res = ref.rotate_back(y3, rot)
    res[:, 0] *= A[t]
    res[:, 1] *= A[t] / wl.h
    res[:, 2] *= A[t] / wl.h
    return res, y[:, 3], f


def test_serve_kernel_and_router():
    wl, px, py, tri, off, idx = mesh_pairs(n_side=48)
    P = idx.numel()
    say(f"serve: pairs={P}")
    p = ref.init_params(5)
    mean, std = np.array([0.2, 0.1, -0.1]), np.array([0.3, 0.5, 0.5])
    A = np.random.default_rng(3).uniform(0.5, 2.0, wl.n_triangles)
    model = sb.surrogate_pack(dev(p), mean, std, 1e30)
    nod = dev(A[None, :])
    # nothing flagged: the network's prediction
    I, Gx, Gy, pp, flags, nf = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx, model, 1e30,
                                                      per_pair=True)
    torch.cuda.synchronize()
    assert int(nf.cpu()) == 0 and int(flags.sum()) == 0
    want, ind, _ = serve_reference(wl, off, idx, p, mean, std, A)
    got = pp.cpu().numpy().T
    for k, name in enumerate(("I", "Gx", "Gy")):
        close_bf16(got[:, k], want[:, k], f"serve {name}")
    # per-particle sums equal the per-pair values summed (FP64 sums of the FP32 network values; only the
    # order of the additions differs from numpy's)
    own = owners(off)
    for k, out in enumerate((I, Gx, Gy)):
        s = np.bincount(own, weights=got[:, k], minlength=wl.n_particles)
        np.testing.assert_allclose(out.cpu().numpy(), s, rtol=1e-13, atol=1e-13 * np.abs(s).max())
    # threshold between indicator values: exactly the pairs above it are flagged
    thr = float(np.median(ind))
    I2, Gx2, Gy2, pp2, flags2, nf2 = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx, model, thr,
                                                            per_pair=True)
    torch.cuda.synchronize()
    fl = flags2.cpu().numpy().astype(bool)
    near = np.abs(ind - thr) < 1e-3 * max(1.0, abs(thr))
    assert np.array_equal(fl[~near], (ind > thr)[~near])
    assert int(nf2.cpu()) == int(fl.sum())
    # flagged pairs carry the closed form, bit for bit equal to the FP64 path's per-pair values
    _, _, _, pp64 = sb.integrate(0, wl.h, px, py, tri, nod, off, idx, per_pair=True)
    got2, ref64 = pp2.cpu().numpy(), pp64.cpu().numpy()
    np.testing.assert_allclose(got2[:, fl], ref64[:, fl], rtol=1e-14, atol=1e-14 * np.abs(ref64).max())
    np.testing.assert_array_equal(got2[:, ~fl], got[~fl].T)
    for k, out in enumerate((I2, Gx2, Gy2)):
        s = np.bincount(own, weights=got2[k], minlength=wl.n_particles)
        np.testing.assert_allclose(out.cpu().numpy(), s, rtol=1e-13, atol=1e-13 * np.abs(s).max())
    # everything flagged: the closed form
    I3, Gx3, Gy3, _, flags3, nf3 = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx, model, -1e30)
    I64, Gx64, Gy64 = sb.integrate(0, wl.h, px, py, tri, nod, off, idx)
    torch.cuda.synchronize()
    assert int(nf3.cpu()) == P
    for a, b in ((I3, I64), (Gx3, Gx64), (Gy3, Gy64)):
        np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-13, atol=1e-13 * float(b.abs().max()))
    # deterministic
    I4, _, _, _, _, _ = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx, model, thr)
    assert torch.equal(I4, I2)


def test_serve_out_of_range_features_are_flagged():
    wl, px, py, tri, off, idx = mesh_pairs(n_side=32)
    p = ref.init_params(6)
    model = sb.surrogate_pack(dev(p), [0, 0, 0], [1, 1, 1], 0.5)      # tiny trained range
    say("serve range")
    nod = dev(np.ones((1, wl.n_triangles)))
    _, _, _, _, flags, nf = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx, model, 1e30)
    own = owners(off)
    f, _ = ref.features(wl.px[own], wl.py[own], wl.tri[:, idx.cpu().numpy()], wl.h)
    out = np.any(np.abs(f[:, :6].astype(np.float32)) > 0.5, axis=1)
    np.testing.assert_array_equal(flags.cpu().numpy().astype(bool), out)
    assert int(nf.cpu()) == int(out.sum())


def test_serve_pairs_outside_the_csr_range_are_not_flagged():
    """Pairs after offsets[-1] belong to no particle: they are never flagged,
    never evaluated, and the results equal those of the exact list."""
    wl, px, py, tri, off, idx = mesh_pairs(n_side=32)
    say("serve stray pairs")
    p = ref.init_params(5)
    model = sb.surrogate_pack(dev(p), [0.2, 0.1, -0.1], [0.3, 0.5, 0.5], 1e30)
    nod = dev(np.ones((1, wl.n_triangles)))
    P = idx.numel()
    stray = torch.as_tensor(np.random.default_rng(2).integers(0, wl.n_triangles, 40).astype(np.int32), device=DEV)
    idx2 = torch.cat([idx, stray])
    for thr in (-1e30, 1e30):
        a = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx, model, thr)
        b = sb.surrogate_integrate(0, wl.h, px, py, tri, nod, off, idx2, model, thr)
        torch.cuda.synchronize()
        for x, y in zip(a[:3], b[:3]):
            assert torch.equal(x, y)
        assert int(b[5].cpu()) == int(a[5].cpu()) == (P if thr < 0 else 0)
        assert int(b[4][P:].sum()) == 0
