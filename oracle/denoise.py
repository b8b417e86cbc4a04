"""Oracle of the learned depth prefilter -- TEST INFRASTRUCTURE ONLY.

Plain numpy (float64 unless a caller passes float32) reference of the small
convolutional encoder-decoder that denoises depth in front of integration,
its masked-L1 loss, the hand-derived backward pass and the Adam update.  Only
tests/, the package smoke check and the benchmark's CPU-baseline leg may use
it; the HIP path never does.

The prefilter is not part of the paper; the nearest thing there is the
optional bilateral filter of the depth input (Sec. 4).  Architecture (one
reading of "4-level 3x3 encoder-decoder with 32/64/64/128 channels"):

  input  x = (d / 4 m, valid mask, hp)                           3 ch, HxW
         hp = (d - mean of the valid depths of the 3x3 neighbourhood) / 5 cm
              on valid pixels, 0 elsewhere
  e1 = relu(conv(x,  3->32,  stride 1))                          H   x W
  e2 = relu(conv(e1, 32->64, stride 2))                          H/2 x W/2
  e3 = relu(conv(e2, 64->64, stride 2))                          H/4 x W/4
  e4 = relu(conv(e3, 64->128, stride 2))                         H/8 x W/8
  d3 = relu(conv(up2(e4), 128->64) + e3)
  d2 = relu(conv(up2(d3), 64->64)  + e2)
  d1 = relu(conv(up2(d2), 64->32)  + e1)
  delta = conv(d1, 32->1)            (zero-initialised weights and bias)
  out = d + 5 cm * delta where d > 0, else 0

conv = 3x3, zero padding 1, with bias; a stride-2 conv samples input pixel
2 o + k - 1 for output o and tap k; up2 = nearest-neighbour upsampling.
Loss = mean over pixels where both the input and the target depth are valid
of |out - target|.  Tensors are NHWC, weights (Cout, 3, 3, Cin).

Parity unpinned: none -- every function here is pinned in
tests/test_oracle_denoise.py (finite differences, a library correlation,
the zero-head identity, Adam's closed form).
"""
from __future__ import annotations

import numpy as np

DEPTH_SCALE = 4.0            # metres: depth input normalisation
CORRECTION_SCALE = 0.05      # metres: the head's output is a correction in units of 5 cm
CHANNELS = (32, 64, 64, 128)
ADAM = dict(lr=2e-4, beta1=0.9, beta2=0.999, eps=1e-8)

# (name, cin, cout, stride, input) of every conv, in forward order
LAYERS = (
    ("e1", 3, 32, 1, "x"),
    ("e2", 32, 64, 2, "e1"),
    ("e3", 64, 64, 2, "e2"),
    ("e4", 64, 128, 2, "e3"),
    ("d3", 128, 64, 1, "up(e4)"),
    ("d2", 64, 64, 1, "up(d3)"),
    ("d1", 64, 32, 1, "up(d2)"),
    ("head", 32, 1, 1, "d1"),
)


def init_params(seed: int = 0, dtype=np.float64) -> dict:
    """He-normal conv weights, zero biases, zero head (identity at start)."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, cin, cout, _, _ in LAYERS:
        if name == "head":
            P[name + ".w"] = np.zeros((cout, 3, 3, cin), dtype)
        else:
            std = np.sqrt(2.0 / (9 * cin))
            P[name + ".w"] = (rng.standard_normal((cout, 3, 3, cin)) * std).astype(dtype)
        P[name + ".b"] = np.zeros(cout, dtype)
    return P


def n_params(P: dict) -> int:
    return int(sum(v.size for v in P.values()))


# ---- building blocks ---------------------------------------------------------------

def out_size(n: int, stride: int) -> int:
    return (n - 1) // stride + 1


def im2col(x: np.ndarray, stride: int) -> np.ndarray:
    """(N, H, W, C) -> (N, Ho, Wo, 3, 3, C): patch of output pixel o, tap
    (ky, kx) = input pixel stride*o + k - 1 (zero outside)."""
    N, H, W, C = x.shape
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((N, H + 2, W + 2, C), x.dtype)
    xp[:, 1:H + 1, 1:W + 1] = x
    cols = np.empty((N, Ho, Wo, 3, 3, C), x.dtype)
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, ky, kx] = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
    return cols


def col2im(cols: np.ndarray, shape, stride: int) -> np.ndarray:
    """adjoint of im2col: scatter-add the patches back to (N, H, W, C)"""
    N, H, W, C = shape
    Ho, Wo = cols.shape[1], cols.shape[2]
    xp = np.zeros((N, H + 2, W + 2, C), cols.dtype)
    for ky in range(3):
        for kx in range(3):
            xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride] += cols[:, :, :, ky, kx]
    return xp[:, 1:H + 1, 1:W + 1]


def conv(x, w, b, stride=1):
    """y[n, o, co] = b[co] + sum_{k, ci} w[co, k, ci] x[n, stride o + k - 1, ci]"""
    cols = im2col(x, stride)
    N, Ho, Wo = cols.shape[:3]
    y = cols.reshape(N * Ho * Wo, -1) @ w.reshape(w.shape[0], -1).T + b
    return y.reshape(N, Ho, Wo, -1)


def conv_backward(x, w, dy, stride=1):
    """(dx, dw, db) of conv for upstream gradient dy"""
    cols = im2col(x, stride)
    N, Ho, Wo = cols.shape[:3]
    dyf = dy.reshape(N * Ho * Wo, -1)
    dw = (dyf.T @ cols.reshape(N * Ho * Wo, -1)).reshape(w.shape)
    db = dyf.sum(axis=0)
    dcols = (dyf @ w.reshape(w.shape[0], -1)).reshape(cols.shape)
    dx = col2im(dcols, x.shape, stride)
    return dx, dw, db


def up2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2)


def up2_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0)


def local_mean(depth):
    """mean of the valid (> 0) depths in each pixel's 3x3 neighbourhood
    (0 where none is valid)"""
    d = np.asarray(depth)
    v = (d > 0).astype(d.dtype)
    N, H, W = d.shape
    dp = np.zeros((N, H + 2, W + 2), d.dtype)
    vp = np.zeros((N, H + 2, W + 2), d.dtype)
    dp[:, 1:H + 1, 1:W + 1] = d * v
    vp[:, 1:H + 1, 1:W + 1] = v
    s = sum(dp[:, ky:ky + H, kx:kx + W] for ky in range(3) for kx in range(3))
    c = sum(vp[:, ky:ky + H, kx:kx + W] for ky in range(3) for kx in range(3))
    return np.where(c > 0, s / np.maximum(c, 1), 0)


def make_input(depth):
    """(N, H, W) metres -> (N, H, W, 3): depth / 4 m, the valid mask, and the
    depth's deviation from its 3x3 valid mean in 5 cm units (valid pixels)"""
    d = np.asarray(depth)
    valid = d > 0
    hp = np.where(valid, (d - local_mean(d)) / CORRECTION_SCALE, 0)
    return np.stack([d / DEPTH_SCALE, valid.astype(d.dtype), hp], axis=-1)


# ---- network ----------------------------------------------------------------------------

def _ident(a):
    return a


def forward(P, depth, q=None):
    """returns (out depth (N, H, W), cache of the activations); H, W divisible
    by 8.  q (default: identity) is applied to the input and to every stored
    activation -- bf16 rounding reproduces the storage precision of the
    matrix-core kernels, so both sides take their relu decisions on the same
    values."""
    q = q or _ident
    dt = P["e1.w"].dtype
    depth = np.asarray(depth, dt)
    x = q(make_input(depth)).astype(dt)
    c = {"x": x, "depth": depth, "q": q}
    c["e1"] = q(relu(conv(x, P["e1.w"], P["e1.b"], 1)))
    c["e2"] = q(relu(conv(c["e1"], P["e2.w"], P["e2.b"], 2)))
    c["e3"] = q(relu(conv(c["e2"], P["e3.w"], P["e3.b"], 2)))
    c["e4"] = q(relu(conv(c["e3"], P["e4.w"], P["e4.b"], 2)))
    c["u4"] = up2(c["e4"])
    c["d3"] = q(relu(conv(c["u4"], P["d3.w"], P["d3.b"]) + c["e3"]))
    c["u3"] = up2(c["d3"])
    c["d2"] = q(relu(conv(c["u3"], P["d2.w"], P["d2.b"]) + c["e2"]))
    c["u2"] = up2(c["d2"])
    c["d1"] = q(relu(conv(c["u2"], P["d1.w"], P["d1.b"]) + c["e1"]))
    c["delta"] = conv(c["d1"], P["head.w"], P["head.b"])[..., 0]
    valid = depth > 0
    out = np.where(valid, depth + CORRECTION_SCALE * c["delta"], 0).astype(dt)
    return out, c


def loss_and_grad_out(out, depth, target):
    """masked L1: mean |out - target| over pixels where depth and target are
    valid; returns (loss, dL/dout, mask count).  The subgradient at 0 is 0."""
    m = (np.asarray(depth) > 0) & (np.asarray(target) > 0)
    n = int(m.sum())
    if n == 0:
        return 0.0, np.zeros_like(out), 0
    diff = out - target
    loss = float(np.abs(diff[m]).sum() / n)
    g = np.where(m, np.sign(diff), 0).astype(out.dtype) / n
    return loss, g, n


def backward(P, c, dout):
    """gradients of every parameter for upstream dL/dout; the gradient at each
    pre-relu sum passes through the forward pass's q (stored like the
    activations)"""
    q = c.get("q", _ident)
    G = {}
    valid = c["depth"] > 0
    ddelta = np.where(valid, CORRECTION_SCALE * dout, 0)[..., None]
    dd1, G["head.w"], G["head.b"] = conv_backward(c["d1"], P["head.w"], ddelta)
    dd1 = q(dd1 * (c["d1"] > 0))                    # through the relu of d1
    du2, G["d1.w"], G["d1.b"] = conv_backward(c["u2"], P["d1.w"], dd1)
    de1_skip = dd1
    dd2 = q(up2_backward(du2) * (c["d2"] > 0))
    du3, G["d2.w"], G["d2.b"] = conv_backward(c["u3"], P["d2.w"], dd2)
    de2_skip = dd2
    dd3 = q(up2_backward(du3) * (c["d3"] > 0))
    du4, G["d3.w"], G["d3.b"] = conv_backward(c["u4"], P["d3.w"], dd3)
    de3_skip = dd3
    de4 = q(up2_backward(du4) * (c["e4"] > 0))
    de3, G["e4.w"], G["e4.b"] = conv_backward(c["e3"], P["e4.w"], de4, 2)
    de3 = q((de3 + de3_skip) * (c["e3"] > 0))
    de2, G["e3.w"], G["e3.b"] = conv_backward(c["e2"], P["e3.w"], de3, 2)
    de2 = q((de2 + de2_skip) * (c["e2"] > 0))
    de1, G["e2.w"], G["e2.b"] = conv_backward(c["e1"], P["e2.w"], de2, 2)
    de1 = q((de1 + de1_skip) * (c["e1"] > 0))
    _, G["e1.w"], G["e1.b"] = conv_backward(c["x"], P["e1.w"], de1)
    return G


def loss_fn(P, depth, target):
    out, _ = forward(P, depth)
    return loss_and_grad_out(out, depth, target)[0]


def adam_step(P, G, state, t, lr=ADAM["lr"], beta1=ADAM["beta1"], beta2=ADAM["beta2"], eps=ADAM["eps"]):
    """one Adam update (Kingma & Ba, Algorithm 1) of every parameter, step t >= 1:
    m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)"""
    for k in P:
        m, v = state.setdefault(k, (np.zeros_like(P[k]), np.zeros_like(P[k])))
        g = G[k]
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
        state[k] = (m, v)


# ---- bfloat16 (round to nearest even), for comparisons with BF16 kernels -------

def to_bf16(a) -> np.ndarray:
    """float32 values rounded to the nearest bfloat16 (ties to even), as float32"""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u >> 16) & 1) + 0x7FFF
    out = ((u + r) >> 16) << 16
    nan = np.isnan(np.asarray(a, np.float32))
    out = out.astype(np.uint32).view(np.float32)
    return np.where(nan, np.float32(np.nan), out)
