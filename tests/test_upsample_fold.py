"""The kernels of an upsampled layer evaluate a nearest 2x upsampling followed
by a 3x3 convolution as four 2x2 convolutions of the source, one per output
parity, on summed weights, each sum carried as two bf16 numbers (hi + lo).
This checks, on the CPU:
* the fold identity in float64 against the oracle's own up2 and conv (plain
  definitions), on ragged sizes, with the tap-to-source-offset rule of the
  kernels' weight packing, and its adjoint against conv_backward + up2_backward;
* that the bf16 split loses nothing where it can be exact: at the offsets one
  or two taps land on, hi + lo equals the exact sum of the bf16 taps whenever
  their float32 sum is exact (the rounding error of a two-term sum is
  representable in the terms' precision), and otherwise (taps more than 2^16
  apart) agrees to float32 resolution; at the four-tap offset to 2^-17
  relative.  So the decoder computes the definition's products up to
  accumulation order."""
import numpy as np

from oracle import denoise as D
from upfold import fold, folded_backward_data, folded_forward, split_fold, taps_per_offset


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


def test_taps_per_offset_are_one_two_two_four():
    n = taps_per_offset()
    for py in range(2):
        for px in range(2):
            assert sorted(n[py, px].reshape(-1).tolist()) == [1, 2, 2, 4]
            # the one-tap offset is (a, b) = (py, px): its low half is zero
            assert n[py, px, py, px] == 1


def test_bf16_split_of_folded_weights_is_exact_up_to_two_taps():
    rng = np.random.default_rng(9)
    # weights spanning several binades, like trained convolution taps
    w = (rng.standard_normal((16, 9, 24)) * np.exp2(rng.integers(-12, 2, (16, 9, 24)))).astype(np.float32)
    s, hi, lo = split_fold(w, D.to_bf16)
    n = np.broadcast_to(taps_per_offset().transpose(0, 1, 2, 3)[:, :, None, :, :, None], s.shape)
    recon = hi.astype(np.float64) + lo.astype(np.float64)
    # the float32 sum of at most two bf16 taps is exact here, and so is hi + lo
    wb = D.to_bf16(w).astype(np.float64)
    exact = fold(wb, np.float64)
    few = n <= 2
    fp32_exact = s.astype(np.float64) == exact
    assert fp32_exact[few].mean() > 0.9
    assert np.array_equal(recon[few & fp32_exact], exact[few & fp32_exact])
    assert np.all(np.abs(recon - exact)[few] <= 2.0 ** -23 * np.abs(exact)[few])
    assert np.all(lo[n == 1] == 0)
    centre = n == 4
    err = np.abs(recon[centre] - s.astype(np.float64)[centre])
    assert np.all(err <= 2.0 ** -17 * np.abs(s.astype(np.float64)[centre]))
    # without the low half the error is a bf16 rounding (about 2^-9)
    assert np.abs(hi.astype(np.float64) - exact)[few].max() > 2.0 ** -12 * np.abs(exact).max()


def test_split_folded_forward_equals_up2_then_3x3_with_bf16_taps():
    rng = np.random.default_rng(10)
    for (N, Hs, Ws, cin, cout) in [(1, 3, 5, 8, 16), (2, 4, 7, 16, 8)]:
        x = D.to_bf16(rng.standard_normal((N, Hs, Ws, cin)).astype(np.float32)).astype(np.float64)
        w = rng.standard_normal((cout, 9, cin)).astype(np.float32)
        b = rng.standard_normal(cout)
        ref = D.conv(D.up2(x), D.to_bf16(w).astype(np.float64), b, 1)
        _, hi, lo = split_fold(w, D.to_bf16)
        got = folded_forward(x, hi.astype(np.float64), b) + folded_forward(x, lo.astype(np.float64), 0.0)
        assert np.allclose(got, ref, rtol=0, atol=2.0 ** -16 * np.abs(ref).max())
