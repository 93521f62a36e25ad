"""Training and serving of the learned surrogate of the per-pair integrals.

The surrogate is an extension, not part of the paper: a small network that
predicts the closed-form per-pair result (I, h Gx, h Gy) of a unit P0 field
for one kernel from the canonical features of the pair (see
``include/sphbi.h``), with an error indicator that routes doubtful pairs back
to the closed form.

This module only orchestrates: the pair lists, the closed-form targets, the
features, the loss gradient, the Adam update and the serving path all run in
the library's kernels.  torch supplies device memory, random batch indices,
summary statistics of the training targets and the calibration of the
router threshold.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (MLP_PARAMS, MLPWorkspace, adam_step, integrate, kernel_preset, mlp_forward, mlp_loss_grad,
               pairlist, surrogate_features, surrogate_integrate, surrogate_pack, surrogate_targets, workloads)

DEV = "cuda:0"


def grad_scale_h(kernel) -> float:
    """h times the natural gradient scale of a unit field: 2 c_d int_0^1 k(q) dq
    (the gradient of a half plane through the particle)."""
    k = kernel_preset(kernel)
    tot = 0.0
    for p in range(k.n_pieces):
        R = k.radius[p]
        tot += sum(k.b[p][j] * R ** (j + 1) / (j + 1) for j in range(k.degree[p] + 1))
    return 2.0 * k.c_d * tot


@dataclass
class PairSet:
    """Pairs of one seeded covering-mesh workload with their closed-form values."""
    feats: torch.Tensor            # float32 [P, 8]
    rot: torch.Tensor              # float32 [P, 2]
    per_pair: torch.Tensor         # float64 [3, P] closed form, unit field (I, Gx, Gy)
    raw: torch.Tensor              # float32 [P, 3] (I, h Gx', h Gy') in the rotated frame
    h: float
    n: int
    geometry: dict = field(default_factory=dict)


def pair_set(seed: int, n_side: int = 1024, kernel: int = 0, keep_geometry: bool = False) -> PairSet:
    """Pairs of a jittered n_side^2 particle grid and a perturbed covering mesh
    (aspect ratio up to 20), h = 2.5 / n_side, unit P0 field."""
    nx, ny = max(1, 128 * n_side // 1024), max(1, 256 * n_side // 1024)
    wl = workloads.covering_workload(n_side=n_side, nx=nx, ny=ny, seed=seed, kernel=kernel, field_order=0)
    px = torch.tensor(wl.px, device=DEV)
    py = torch.tensor(wl.py, device=DEV)
    tri = torch.tensor(wl.tri, device=DEV)
    nod = torch.ones((1, wl.n_triangles), dtype=torch.float64, device=DEV)
    off, idx = pairlist(px, py, tri, wl.h)
    _, _, _, pp = integrate(kernel, wl.h, px, py, tri, nod, off, idx, per_pair=True)
    feats, rot = surrogate_features(px, py, tri, wl.h, off, idx)
    raw = surrogate_targets(pp, rot, wl.h)
    geo = dict(px=px, py=py, tri=tri, off=off, idx=idx, nodal=nod) if keep_geometry else {}
    return PairSet(feats, rot, pp, raw, wl.h, int(idx.numel()), geo)


def init_params(seed: int) -> torch.Tensor:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and zero biases (FP32 master copy)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for fin, fout in ((8, 128), (128, 128), (128, 128), (128, 4)):
        lim = 1.0 / math.sqrt(fin)
        parts.append((torch.rand(fin * fout, generator=g, dtype=torch.float64) * 2 - 1) * lim)
        parts.append(torch.zeros(fout, dtype=torch.float64))
    p = torch.cat(parts).float()
    assert p.numel() == MLP_PARAMS
    return p.to(DEV)


class Surrogate:
    """FP32 master weights, Adam state and output statistics of one trained network."""

    def __init__(self, kernel: int = 0, seed: int = 0):
        self.kernel = kernel
        self.params = init_params(seed)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.mean = np.zeros(3)
        self.stdev = np.ones(3)
        self.fmax = 0.0
        self.threshold = float("inf")
        self.sg = grad_scale_h(kernel)

    # -------------------------------------------------------------- training
    def fit_statistics(self, sets):
        raw = torch.cat([s.raw for s in sets]).double()
        self.mean = raw.mean(0).cpu().numpy()
        self.stdev = raw.std(0).cpu().numpy()
        self.fmax = float(max(float(s.feats[:, :6].abs().max()) for s in sets))

    def err_scale(self):
        """standardised units -> scale-normalised error (I: 1, h G: 2 c_d int k)"""
        return [self.stdev[0], self.stdev[1] / self.sg, self.stdev[2] / self.sg]

    def train(self, sets, steps: int, batch: int = 16384, lr: float = 2e-3, lr_min: float = 2e-5,
              lam: float = 0.05, seed: int = 1, log=None, log_every: int = 500):
        """Adam on the mean squared error of the standardised targets plus the
        indicator term, with a cosine learning-rate decay over `steps`."""
        if self.step == 0:
            self.fit_statistics(sets)
        feats = torch.cat([s.feats for s in sets])
        tgt = torch.cat([surrogate_targets(s.per_pair, s.rot, s.h, self.mean, self.stdev) for s in sets])
        P = feats.shape[0]
        ws = MLPWorkspace(batch)
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=DEV)
        loss = torch.empty(1, dtype=torch.float32, device=DEV)
        gen = torch.Generator(device=DEV).manual_seed(seed + self.step)
        scale = self.err_scale()
        t0 = time.perf_counter()
        first = self.step
        history = []
        for k in range(steps):
            b = torch.randint(0, P, (batch,), device=DEV, generator=gen)
            x, t = feats.index_select(0, b), tgt.index_select(0, b)
            mlp_loss_grad(self.params, x, t, scale, lam, ws=ws, grad=grad, loss=loss)
            frac = k / max(1, steps - 1)
            lr_k = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * frac))
            self.step += 1
            adam_step(self.params, self.m, self.v, grad, lr_k, self.step)
            if log is not None and (k % log_every == 0 or k == steps - 1):
                lv = float(loss.item())
                history.append((self.step, lv))
                log(f"  step {self.step} loss {lv:.4e} lr {lr_k:.2e} ({time.perf_counter() - t0:.1f} s)")
        torch.cuda.synchronize()
        return {"steps": self.step - first, "seconds": time.perf_counter() - t0, "pairs": P, "history": history}

    # -------------------------------------------------------------- evaluation
    def predict(self, feats, chunk: int = 1 << 20):
        """Network outputs [P, 4] (standardised, rotated frame; indicator last)."""
        ws = MLPWorkspace(min(chunk, feats.shape[0]))
        return torch.cat([mlp_forward(self.params, feats[i:i + chunk], ws=ws)
                          for i in range(0, feats.shape[0], chunk)])

    def pair_errors(self, s: PairSet, out=None):
        """(scale-normalised error of every pair, indicator) of the unrouted network."""
        out = self.predict(s.feats) if out is None else out
        t = surrogate_targets(s.per_pair, s.rot, s.h, self.mean, self.stdev)
        sc = torch.tensor(self.err_scale(), device=DEV, dtype=torch.float32)
        err = ((out[:, :3] - t).abs() * sc).max(1).values
        return err, out[:, 3]

    def calibrate(self, s: PairSet, level: float, miss: float = 1e-4):
        """Largest threshold such that, among the calibration pairs whose
        indicator is at or below it, at most a fraction `miss` has a
        scale-normalised error above `level`."""
        err, ind = self.pair_errors(s)
        order = torch.argsort(ind)
        viol = torch.cumsum((err[order] > level).double(), 0)
        k = torch.arange(1, order.numel() + 1, device=viol.device, dtype=torch.float64)
        ok = torch.nonzero(viol <= miss * k)
        if ok.numel() == 0:
            self.threshold = float("-inf")
            return self.threshold
        j = int(ok.max())
        if j + 1 >= order.numel():
            self.threshold = float("inf")
        else:
            # just below the first indicator value that is not accepted
            nxt = np.float32(ind[order[j + 1]].item())
            self.threshold = float(np.nextafter(nxt, np.float32(-np.inf)))
        return self.threshold

    # -------------------------------------------------------------- serving
    def model(self):
        return surrogate_pack(self.params, self.mean, self.stdev, self.fmax)

    def integrate(self, h, px, py, tri, nodal, offsets, tri_idx, model=None, threshold=None, per_pair=False, ws=None):
        model = self.model() if model is None else model
        thr = self.threshold if threshold is None else threshold
        return surrogate_integrate(self.kernel, h, px, py, tri, nodal, offsets, tri_idx, model, thr,
                                   per_pair=per_pair, ws=ws)

    # -------------------------------------------------------------- checkpoint
    def state_dict(self):
        return {"kernel": self.kernel, "params": self.params.cpu(), "m": self.m.cpu(), "v": self.v.cpu(),
                "step": self.step, "mean": torch.tensor(self.mean), "stdev": torch.tensor(self.stdev),
                "fmax": self.fmax, "threshold": self.threshold}

    def save(self, path):
        torch.save(self.state_dict(), path)

    @classmethod
    def load(cls, path):
        d = torch.load(path, weights_only=True)
        s = cls(kernel=int(d["kernel"]))
        s.params = d["params"].to(DEV)
        s.m = d["m"].to(DEV)
        s.v = d["v"].to(DEV)
        s.step = int(d["step"])
        s.mean = d["mean"].numpy()
        s.stdev = d["stdev"].numpy()
        s.fmax = float(d["fmax"])
        s.threshold = float(d["threshold"])
        return s
