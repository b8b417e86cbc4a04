"""The forward kernel of an upsampled layer evaluates a nearest 2x upsampling
followed by a 3x3 convolution as four 2x2 convolutions of the source, one per
output parity, on summed weights.  This checks that identity in float64
against the oracle's own up2 and conv (plain definitions), on ragged sizes,
with the tap-to-source-offset rule the kernel's weight packing uses."""
import numpy as np

from oracle import denoise as D
from upfold import fold, folded_backward_data, folded_forward


def test_each_tap_lands_on_one_of_two_source_offsets():
    for p in range(2):
        offs = [((p + k - 1) >> 1) + 1 - p for k in range(3)]
        assert sorted(set(offs)) == [0, 1]
        # the source offset of tap k is floor((p + k - 1) / 2) relative to row m
        assert [o + p - 1 for o in offs] == [(p + k - 1) // 2 for k in range(3)]


def test_parity_folded_2x2_equals_up2_then_3x3():
    rng = np.random.default_rng(7)
    for (N, Hs, Ws, cin, cout) in [(1, 1, 1, 2, 3), (2, 3, 5, 3, 4), (1, 4, 7, 8, 16)]:
        x = rng.standard_normal((N, Hs, Ws, cin))
        w = rng.standard_normal((cout, 9, cin))
        b = rng.standard_normal(cout)
        ref = D.conv(D.up2(x), w, b, 1)
        got = folded_forward(x, fold(w), b)
        assert got.shape == ref.shape
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12), (N, Hs, Ws, np.abs(got - ref).max())


def test_folded_adjoint_equals_conv_backward_then_up2_backward():
    rng = np.random.default_rng(8)
    for (N, Hs, Ws, cin, cout) in [(1, 1, 1, 2, 3), (2, 3, 5, 3, 4), (1, 4, 7, 8, 16)]:
        x = rng.standard_normal((N, Hs, Ws, cin))
        w = rng.standard_normal((cout, 3, 3, cin))
        g = rng.standard_normal((N, 2 * Hs, 2 * Ws, cout))
        dx, _, _ = D.conv_backward(D.up2(x), w, g, 1)
        ref = D.up2_backward(dx)
        got = folded_backward_data(g, fold(w))
        assert got.shape == ref.shape
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12), (N, Hs, Ws, np.abs(got - ref).max())
