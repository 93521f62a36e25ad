"""CPU reference of the learned surrogate -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  Plain NumPy in float64, written from the
definitions; it shares no code with the device kernels.

The surrogate is not part of the paper: it approximates the per-pair result
of the paper's boundary integral (Sec. 2, eq. boundaryint with a unit field
and eq. nablaIntegral) for Wendland C2 in the support-normalised particle
frame of Sec. 2 (transform C).

Features (per pair, h-frame, coordinates nu = (v - x)/h):
  * the triangle is put in counter-clockwise order (the integrals do not
    depend on orientation), its vertices cyclically shifted so that the one
    nearest the particle comes first (lowest index on ties), and the frame
    rotated about the particle so that this vertex lies on the +x axis
    (identity when it coincides with the particle);
  * features 0-5: the three rotated vertices; feature 6: the number of
    vertices with |nu| <= 1, over 3; feature 7: the number of edges whose
    segment meets the circle |nu| = 1, over 3.
The outputs (I, h Gx, h Gy) are predicted in the rotated frame; the gradient
is rotated back.  Every geometric decision is taken in float64 without fused
multiply-adds, as in the device code.

Network: 8 -> 128 -> 128 -> 128 -> 4, activation act() between layers.  Outputs 0-2 are the
standardised targets, output 3 an error indicator trained on the log10 of the
network's own (detached) scaled error.  Parameters are one flat float32
vector: W1[8][128], b1, W2[128][128], b2, W3[128][128], b3, W4[128][4], b4.

Loss of a batch of B pairs (mean over the batch):
  L = sum_k (y_k - t_k)^2 / (3B) + lam * (y_3 - e)^2 / B,
  e = log10(max_k |y_k - t_k| s_k + 1e-7), with e detached (no gradient),
where s_k converts standardised units back to the scale-normalised error.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(8, 128), (128, 128), (128, 128), (128, 4)]
N_PARAMS = sum(i * o + o for i, o in LAYERS)      # 34,692
ERR_FLOOR = 1e-7


# ----------------------------------------------------------------------------
# bfloat16 rounding (round to nearest even from float32), as the device does
# ----------------------------------------------------------------------------
def bf16(x):
    """Round to bfloat16 through float32 (returns float64)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------
def features(px, py, tri, h):
    """Canonical features of pairs.

    px, py: [P] particle positions; tri: [6, P] vertex coordinates of each
    pair's triangle (x0, y0, x1, y1, x2, y2).  Returns (feats [P, 8],
    rot [P, 2] = (cos, sin) of the frame rotation).
    """
    px = np.asarray(px, np.float64)
    py = np.asarray(py, np.float64)
    tri = np.asarray(tri, np.float64)
    P = px.shape[0]
    ih = 1.0 / h
    feats = np.zeros((P, 8))
    rot = np.zeros((P, 2))
    for q in range(P):
        v = [((tri[2 * k, q] - px[q]) * ih, (tri[2 * k + 1, q] - py[q]) * ih) for k in range(3)]
        area2 = (v[1][0] - v[0][0]) * (v[2][1] - v[0][1]) - (v[2][0] - v[0][0]) * (v[1][1] - v[0][1])
        if area2 < 0.0:
            v = [v[0], v[2], v[1]]
        d2 = [a * a + b * b for a, b in v]
        first = 0
        for k in (1, 2):
            if d2[k] < d2[first]:
                first = k
        v = [v[(first + k) % 3] for k in range(3)]
        r = np.sqrt(d2[first])
        c, s = (v[0][0] / r, v[0][1] / r) if r > 0.0 else (1.0, 0.0)
        w = [(c * a + s * b, c * b - s * a) for a, b in v]
        inside = sum(1 for a, b in v if a * a + b * b <= 1.0)
        cross = sum(1 for k in range(3) if _segment_meets_circle(v[k], v[(k + 1) % 3]))
        feats[q] = [w[0][0], w[0][1], w[1][0], w[1][1], w[2][0], w[2][1], inside / 3.0, cross / 3.0]
        rot[q] = (c, s)
    return feats, rot


def _segment_meets_circle(a, b):
    """Whether the segment a-b has a point with |x| = 1 (exact case analysis)."""
    da = a[0] * a[0] + a[1] * a[1]
    db = b[0] * b[0] + b[1] * b[1]
    if (da <= 1.0) != (db <= 1.0):
        return True
    if da <= 1.0:                  # both inside
        return False
    # both outside: does the closest point of the segment lie inside?
    ex, ey = b[0] - a[0], b[1] - a[1]
    L2 = ex * ex + ey * ey
    if L2 == 0.0:
        return False
    t = -(a[0] * ex + a[1] * ey) / L2
    if t <= 0.0 or t >= 1.0:
        return False
    cx, cy = a[0] + t * ex, a[1] + t * ey
    return cx * cx + cy * cy < 1.0


def rotate_back(y, rot):
    """Map predictions (I, hGx', hGy') of the rotated frame to the h-frame."""
    c, s = rot[:, 0], rot[:, 1]
    out = np.array(y[:, :3], dtype=np.float64, copy=True)
    out[:, 1] = c * y[:, 1] - s * y[:, 2]
    out[:, 2] = s * y[:, 1] + c * y[:, 2]
    return out


def rotate_in(t, rot):
    """Express (I, hGx, hGy) of the h-frame in the rotated frame."""
    c, s = rot[:, 0], rot[:, 1]
    out = np.array(t, dtype=np.float64, copy=True)
    out[:, 1] = c * t[:, 1] + s * t[:, 2]
    out[:, 2] = -s * t[:, 1] + c * t[:, 2]
    return out


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------
def unpack(params):
    """Flat parameter vector -> [(W [in, out], b [out])] per layer."""
    params = np.asarray(params, np.float64)
    out, o = [], 0
    for i, n in LAYERS:
        W = params[o:o + i * n].reshape(i, n)
        o += i * n
        b = params[o:o + n]
        o += n
        out.append((W, b))
    return out


def act(z):
    """z s(z) with s(z) = 1/2 + u/4 - u|u|/32, u = clamp(z, -4, 4): a
    continuously differentiable piecewise quadratic stand-in for
    z sigmoid(z) (s rises from 0 at z = -4 to 1 at z = 4 with zero slope at
    both ends)."""
    z = np.asarray(z, np.float64)
    u = np.clip(z, -4.0, 4.0)
    return z * (0.5 + u * (0.25 - np.abs(u) / 32.0))


def act_grad(z):
    z = np.asarray(z, np.float64)
    inner = 0.5 + z * (0.5 - 3.0 * np.abs(z) / 32.0)
    return np.where(z >= 4.0, 1.0, np.where(z <= -4.0, 0.0, inner))


def split_bf16(x):
    """x (float32) as hi + lo with hi = bf16(x), lo = bf16(x - hi): the
    network's first layer sees its inputs to about 16 significant bits."""
    x = np.asarray(x, np.float32).astype(np.float64)
    hi = bf16(x)
    return hi + bf16(x - hi)


def forward(params, x, round_bf16=False):
    """Network outputs [B, 4]; with round_bf16 the weights and every layer
    input are rounded to bfloat16 (the features to a pair of bfloat16
    numbers, see split_bf16; products and sums stay exact)."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    a = split_bf16(x) if round_bf16 else np.asarray(x, np.float64)
    layers = unpack(params)
    for li, (W, b) in enumerate(layers):
        z = a @ r(W) + b
        a = r(act(z)) if li < len(layers) - 1 else z
    return a


def loss_and_grad(params, x, t, scale, lam, round_bf16=False):
    """Batch loss and its gradient with respect to the flat parameters.

    x [B, 8] features, t [B, 3] standardised targets, scale [3] the factors
    s_k.  Backward by the chain rule through the same (optionally rounded)
    operands as the forward pass (with round_bf16 the pre-activation
    gradients are rounded too before they enter the products); the indicator
    target e is a constant.
    """
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    B = x.shape[0]
    layers = unpack(params)
    acts = [split_bf16(x) if round_bf16 else np.asarray(x, np.float64)]
    zs = []
    for li, (W, b) in enumerate(layers):
        z = acts[-1] @ r(W) + b
        zs.append(z)
        if li < len(layers) - 1:
            acts.append(r(act(z)))
    y = zs[-1]
    d = y[:, :3] - t
    e = np.log10(np.max(np.abs(d) * scale, axis=1) + ERR_FLOOR)
    L = np.sum(d * d) / (3 * B) + lam * np.sum((y[:, 3] - e) ** 2) / B
    dz = np.zeros_like(y)
    dz[:, :3] = 2.0 * d / (3 * B)
    dz[:, 3] = 2.0 * lam * (y[:, 3] - e) / B
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in = acts[li]
        dzr = r(dz)                 # the products take rounded operands
        gW = a_in.T @ dzr
        gb = dzr.sum(0)
        grads.append((gW, gb))
        if li > 0:
            da = dzr @ r(W).T
            dz = da * act_grad(zs[li - 1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam(params, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) with bias correction; returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights, zero biases, as float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, n in LAYERS:
        lim = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-lim, lim, size=i * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)
