"""The paper's synthetic studies at full scale on the device.

Signal degradation (Sec. 4): the band at 73 degrees carried across the
hole at 200 x 100 ... 8000 x 4000; the device fill matches the oracle at
every resolution (shell maps bit-exact; colours within 1e-5 relative, or K
binary32 roundings for the deep fills of K = 600 and 1200 shells), its shells are the hole's chessboard rings, and the error over
the hole falls at least like h^(1/(2p)) (eqn:Lpbound).

Camera-pan video (the frame-by-frame film workload of Sec. 7): every frame is
a window of one static scene; with the holes kept away from the frame
borders the fill of a scene pixel cannot depend on where the window sits, so
one batched launch must give bit-identical colours and shells for a scene
pixel in every frame that shows it."""

import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synthetic as syn
from gpu_helpers import assert_colour_parity, banner, gpu_fill

pytestmark = pytest.mark.gpu

LAUNCH = {"tiled": {}, "front": {"engine": 1}}


def _lp(u, prob, p):
    e = np.abs(u - prob.exact)[prob.label == 1]
    return (prob.h * prob.h * (e ** p).sum()) ** (1.0 / p)


@pytest.mark.parametrize("W", [200, 400, 4000, 8000])
def test_degradation_parity_and_shells(W):
    banner(f"degradation {W}x{W // 2}")
    prob = syn.degradation_problem(W)
    ref = oracle.fill(prob.image, prob.label, prob.guide, eps=3.0, mu=50.0)
    engines = ["tiled", "front"] if W <= 400 else ["tiled"]
    d = ndimage.distance_transform_cdt(prob.label == 1, metric="chessboard")
    for eng in engines:
        u, s, st, _ = gpu_fill(prob.image, prob.label, prob.guide, **LAUNCH[eng])
        np.testing.assert_array_equal(s, ref.shell)
        np.testing.assert_array_equal(np.where(prob.label == 1, s, -1),
                                      np.where(prob.label == 1, d - 1, -1))
        assert st["K"] == int(d.max())
        # each shell reads the last shells' binary32 values: one rounding
        # (2^-24 relative) per shell can add up along the K dependent shells
        assert_colour_parity(u, ref.u, s, tol=max(1e-5, st["K"] * 2.0 ** -24))


def test_degradation_rate_at_scale():
    """L^1 and L^2 errors over the hole from 200 x 100 to 8000 x 4000: each
    doubling of the resolution lowers them at least by 2^(0.9 / (2p))."""
    banner("degradation rates")
    errs = {1: [], 2: []}
    Ws = [200, 400, 800, 1600, 4000, 8000]
    for W in Ws:
        prob = syn.degradation_problem(W)
        u, s, st, _ = gpu_fill(prob.image, prob.label, prob.guide)
        assert st["unfilled"] == 0
        for p in (1, 2):
            errs[p].append(_lp(u[..., 0].astype(np.float64), prob, p))
    print("L1", [f"{e:.5f}" for e in errs[1]], "L2", [f"{e:.5f}" for e in errs[2]], flush=True)
    for p in (1, 2):
        for (wa, ea), (wb, eb) in zip(zip(Ws, errs[p]), zip(Ws[1:], errs[p][1:])):
            rate = math.log(ea / eb) / math.log(wb / wa)
            assert rate >= 0.9 / (2 * p), (p, wa, wb, rate)


@pytest.mark.parametrize("engine", ["tiled", "front"])
def test_pan_video_is_translation_exact(engine):
    banner(f"pan video {engine}")
    B, H, W, step = 6, 270, 480, (5, 2)
    wl, origins = syn.pan_video(seed=6, B=B, H=H, W=W, step=step, dtype=np.float32)
    assert (wl.label == 1).sum() > 0
    u, s, st, _ = gpu_fill(wl.image, wl.label, wl.guide, **LAUNCH[engine])
    # the scene pixels every frame shows: the window of the last frame's origin
    # intersected with the first one's
    x0, y0 = origins[-1]
    cw, ch = W - x0, H - y0
    ref_u = u[0][y0:y0 + ch, x0:x0 + cw]
    ref_s = s[0][y0:y0 + ch, x0:x0 + cw]
    for t, (ox, oy) in enumerate(origins):
        ut = u[t][y0 - oy:y0 - oy + ch, x0 - ox:x0 - ox + cw]
        stt = s[t][y0 - oy:y0 - oy + ch, x0 - ox:x0 - ox + cw]
        np.testing.assert_array_equal(stt, ref_s)
        np.testing.assert_array_equal(ut, ref_u)
    # and frame 0 against the oracle
    r0 = oracle.fill(wl.image[0], wl.label[0], wl.guide[0], eps=3.0, mu=50.0)
    np.testing.assert_array_equal(s[0], r0.shell)
    assert_colour_parity(u[0], r0.u, s[0], tol=1e-5)
