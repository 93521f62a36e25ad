"""Error measures for comparing device results with the oracle.

The scale-normalised error e = |y - y_ref| / max(|y_ref|, S) uses the natural
scale of each output: S_I = max|A| (the integral over a full support disc of
a unit field is 1) and S_G = 2 c_d int_0^1 k dq / h * max|A| (the gradient of a
half plane through the particle).  Values near zero make a pure relative
error meaningless, so this is the measure the tolerances refer to.
"""
import numpy as np

from tests import exact


def grad_scale(kid, h):
    return float(2 * exact.c_d(kid) * exact.int_k(kid)) / h


def scaled_err(got, ref, scale):
    got, ref = np.asarray(got), np.asarray(ref)
    return np.abs(got - ref) / np.maximum(np.abs(ref), scale)


def report(kid, h, amax, got, ref):
    """Max scale-normalised errors of (I, Gx, Gy)."""
    sI = max(amax, 1e-300)
    sG = grad_scale(kid, h) * max(amax, 1e-300)
    eI = scaled_err(got[0], ref[0], sI)
    eG = np.maximum(scaled_err(got[1], ref[1], sG), scaled_err(got[2], ref[2], sG))
    return float(eI.max(initial=0.0)), float(eG.max(initial=0.0))
