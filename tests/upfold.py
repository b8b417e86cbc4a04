"""Test helper: a nearest 2x upsampling followed by a 3x3 convolution written
as four 2x2 convolutions of the source, one per output parity (py, px).  Tap
ky lands on source row offset a = floor((py + ky - 1) / 2) + 1 - py in {0, 1}
(likewise kx -> b), so output (2m + py, 2n + px) reads source pixels
(m + py - 1 + a, n + px - 1 + b)."""
import numpy as np


def fold(w, acc_dtype=np.float64):
    """(cout, 3, 3, cin) or (cout, 9, cin) -> (2, 2, cout, 2, 2, cin):
    [py][px][co][a][b][ci], summed in ascending (ky, kx) order in `acc_dtype`"""
    w = w.reshape(w.shape[0], 9, w.shape[-1])
    cout, _, cin = w.shape
    f = np.zeros((2, 2, cout, 2, 2, cin), acc_dtype)
    for py in range(2):
        for px in range(2):
            for ky in range(3):
                a = ((py + ky - 1) >> 1) + 1 - py
                for kx in range(3):
                    b = ((px + kx - 1) >> 1) + 1 - px
                    f[py, px, :, a, b, :] += w[:, ky * 3 + kx, :].astype(acc_dtype)
    return f


def folded_forward(x, f, bias):
    """(N, Hs, Ws, cin) source, folded weights -> (N, 2 Hs, 2 Ws, cout), no relu"""
    N, Hs, Ws, cin = x.shape
    cout = f.shape[2]
    xp = np.zeros((N, Hs + 2, Ws + 2, cin))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((N, 2 * Hs, 2 * Ws, cout))
    for py in range(2):
        for px in range(2):
            acc = np.zeros((N, Hs, Ws, cout)) + bias
            for a in range(2):
                for b in range(2):
                    src = xp[:, py + a:py + a + Hs, px + b:px + b + Ws]
                    acc += src @ f[py, px, :, a, b, :].astype(np.float64).T
            y[:, py::2, px::2] = acc
    return y


def folded_backward_data(g, f):
    """gradient at the (N, Hs, Ws, cin) source of folded_forward for the
    upstream gradient g (N, 2 Hs, 2 Ws, cout): source pixel (m, n) collects
    output (2 m' + py, 2 n' + px) with m' = m + 1 - py - a, n' = n + 1 - px - b"""
    N, Ho, Wo, cout = g.shape
    Hs, Ws = Ho // 2, Wo // 2
    cin = f.shape[-1]
    dx = np.zeros((N, Hs + 2, Ws + 2, cin))
    for py in range(2):
        for px in range(2):
            gp = g[:, py::2, px::2]   # (N, Hs, Ws, cout) at m', n'
            for a in range(2):
                for b in range(2):
                    # output m' feeds source m' + py - 1 + a (padded index + 1)
                    dx[:, py + a:py + a + Hs, px + b:px + b + Ws] += gp @ f[py, px, :, a, b, :].astype(np.float64)
    return dx[:, 1:-1, 1:-1]


def split_fold(w, to_bf16):
    """the decoder kernels' weight operands: the fold of the bf16-rounded
    taps summed in float32 (ascending ky, kx), then split into bf16 halves
    hi = bf16(s), lo = bf16(s - hi).  Returns (s, hi, lo), float32 arrays of
    fold's shape; `to_bf16` rounds float32 to bf16 values (nearest even)."""
    wb = to_bf16(np.asarray(w, np.float32))
    s = fold(wb, np.float32)
    hi = to_bf16(s)
    lo = to_bf16((s - hi).astype(np.float32))
    return s, hi, lo


def taps_per_offset():
    """(2, 2, 2, 2) counts of the 3x3 taps landing on source offset (a, b)
    for output parity (py, px)"""
    return fold(np.ones((1, 9, 1))).reshape(2, 2, 2, 2)
