"""FP64 CPU reference of the learned scheduler's CNN (test infrastructure only).

Same layout as the GPU model: grid of D x H x W voxels, channels last; three
3x3x3 convolutions with zero padding (3 -> C -> C -> 1 channels), ReLU after
the first two, logits out; binary cross-entropy with logits averaged over the
masked voxels.  Parameters (flat): w1[C][3][27] b1[C] w2[C][C][27] b2[C]
w3[1][C][27] b3[1], tap = (dz+1)*9 + (dy+1)*3 + (dx+1).

This is the textbook definition written out with explicit taps; the tests pin
the convolution against scipy's correlation and the gradients against central
finite differences.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def num_params(C):
    return C * 3 * 27 + C + C * C * 27 + C + C * 27 + 1


def unpack(p, C):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("w1", (C, 3, 27)), ("b1", (C,)), ("w2", (C, C, 27)), ("b2", (C,)),
                        ("w3", (1, C, 27)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    assert o == p.size
    return out


def pack(d):
    return np.concatenate([d[k].reshape(-1) for k in ("w1", "b1", "w2", "b2", "w3", "b3")])


def _shift(x, dz, dy, dx):
    """s[z,y,x] = x[z+dz, y+dy, x+dx] (zero outside), over the first three axes."""
    D, H, W = x.shape[:3]
    s = np.zeros_like(x)
    zs = slice(max(0, -dz), min(D, D - dz))
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    zt = slice(max(0, dz), min(D, D + dz))
    yt = slice(max(0, dy), min(H, H + dy))
    xt = slice(max(0, dx), min(W, W + dx))
    s[zs, ys, xs] = x[zt, yt, xt]
    return s


def conv3(x, w, b):
    """y[v, co] = b[co] + sum_ci sum_tap w[co, ci, tap] x[v + tap, ci]."""
    y = np.broadcast_to(b, x.shape[:3] + (w.shape[0],)).copy()
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += _shift(x, dz, dy, dx) @ w[:, :, t].T
    return y


def conv3_backward(x, w, gy):
    """Gradients of sum(gy * conv3(x, w, b)) w.r.t. x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = _shift(x, dz, dy, dx)
        gw[:, :, t] = np.einsum("zyxo,zyxi->oi", gy, xs)
        gx += _shift(gy @ w[:, :, t], -dz, -dy, -dx)
    gb = gy.sum(axis=(0, 1, 2))
    return gx, gw, gb


def forward(p, x, C):
    """x: [D, H, W, 3] (extra feature channels are ignored). Returns logits [D,H,W] and a cache."""
    q = unpack(p, C)
    x = np.asarray(x, dtype=np.float64)[..., :3]
    a1 = conv3(x, q["w1"], q["b1"])
    h1 = np.maximum(a1, 0.0)
    a2 = conv3(h1, q["w2"], q["b2"])
    h2 = np.maximum(a2, 0.0)
    z = conv3(h2, q["w3"], q["b3"])[..., 0]
    return z, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, q=q)


def bce_loss(z, t, m):
    z = np.asarray(z, np.float64)
    t = np.asarray(t, np.float64)
    m = np.asarray(m, np.float64)
    tot = m.sum()
    per = np.maximum(z, 0) - z * t + np.log1p(np.exp(-np.abs(z)))
    loss = float((per * m).sum() / tot) if tot > 0 else 0.0
    gz = (1.0 / (1.0 + np.exp(-z)) - t) * m / tot if tot > 0 else np.zeros_like(z)
    return loss, gz


def loss_and_grad(p, x, t, m, C):
    z, c = forward(p, x, C)
    loss, gz = bce_loss(z, t, m)
    q = c["q"]
    gh2, gw3, gb3 = conv3_backward(c["h2"], q["w3"], gz[..., None])
    ga2 = gh2 * (c["a2"] > 0)
    gh1, gw2, gb2 = conv3_backward(c["h1"], q["w2"], ga2)
    ga1 = gh1 * (c["a1"] > 0)
    _, gw1, gb1 = conv3_backward(c["x"], q["w1"], ga1)
    return loss, pack(dict(w1=gw1, b1=gb1, w2=gw2, b2=gb2, w3=gw3, b3=gb3))


def bf16_round(x):
    """Round float32 values to bfloat16 (8 significant bits, ties to even),
    kept as float32.  Written from the definition: split x = m * 2^e with
    0.5 <= |m| < 1, scale the significand to 8 bits, round half to even
    (np.rint), scale back.  Finite inputs."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8).astype(np.float32)


def conv3_bf16(x, w, b):
    """The bf16 form of conv3: x and w are bfloat16 values (already rounded),
    the bias is float32, and every sum is a float32 sum taken in one fixed
    order: the bias, then the taps in TAPS order, and within a tap the input
    channels in increasing order.  A product of two bfloat16 values is exact in
    float32, so this order fixes every bit of the result."""
    x = np.asarray(x, dtype=np.float32)
    w = np.asarray(w, dtype=np.float32)
    cout, cin = w.shape[0], w.shape[1]
    y = np.empty(x.shape[:3] + (cout,), np.float32)
    y[...] = np.asarray(b, dtype=np.float32)
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = _shift(x, dz, dy, dx)
        for ci in range(cin):
            y += xs[..., ci:ci + 1] * w[:, ci, t]
    return y


def forward_bf16(p, x, C):
    """Logits of the bf16 inference path: inputs and weights rounded to
    bfloat16, float32 sums (conv3_bf16), ReLU, and every layer's output
    rounded to bfloat16."""
    q = unpack(p, C)
    r = lambda a: bf16_round(np.asarray(a, np.float32))
    x = r(np.asarray(x, np.float32)[..., :3])
    h1 = r(np.maximum(conv3_bf16(x, r(q["w1"]), q["b1"]), 0.0))
    h2 = r(np.maximum(conv3_bf16(h1, r(q["w2"]), q["b2"]), 0.0))
    return r(conv3_bf16(h2, r(q["w3"]), q["b3"]))[..., 0]
