"""The evaluation on the GPU compares like with like: fused through a
prefilter that is the identity (a zero head), a held-out room gives exactly
the raw path's surface RMS and hit counts at every frame count, so the
equal-error comparison of the two paths reaches e* at the last N with
equal errors; and more frames lower the raw path's RMS on noisy depth."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_identity_prefilter_evaluates_like_raw_depth():
    import torch
    import paper_1708_00783_amd as T
    from paper_1708_00783_amd import prefilter as PF
    from synth import configs
    n = 30
    frames = torch.from_numpy(np.stack([configs.c2_frame(k, 6000) for k in range(n)])).cuda()
    net = T.Denoiser(1, 480, 640)
    net.set_params(PF.init_params(0))           # zero head: the identity on valid pixels
    strides = (10, 3, 1)
    raw = PF.evaluate_room(6000, frames, None, strides=strides)
    den = PF.evaluate_room(6000, frames, net, strides=strides)
    ns = sorted(raw)
    assert ns == [3, 10, 30]
    for k in ns:
        assert raw[k][0] == den[k][0] and raw[k][2] == den[k][2], (k, raw[k], den[k])
    e, nd, _ = PF.equal_error(ns, [raw[k][0] for k in ns], [den[k][0] for k in ns], [raw[k][2] for k in ns],
                              [den[k][2] for k in ns], [raw[k][1] for k in ns], [den[k][1] for k in ns])
    assert nd == 30 and e == raw[30][0]
    assert raw[30][0] < raw[3][0]
    print(f"raw RMS by frames fused: {[(k, round(raw[k][0] * 1e3, 3)) for k in ns]} mm", flush=True)
