"""The guide field of Sec. 3.2 on the device (gf_guide_field) against the
oracle's construction, on seeded random polylines: identical choice of spline
and cutoff (FP64 on both sides), values within 1e-6 (the GPU rounds the result
to binary32; exp differs by at most an ulp in FP64)."""

import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _gpu(label, seg, off, eta=3.0, cutoff=None):
    import torch

    import paper_1611_05319_amd as gf

    dev = torch.device("cuda:0")
    lab = torch.from_numpy(np.ascontiguousarray(label)).to(dev)
    sg = torch.from_numpy(np.ascontiguousarray(seg, dtype=np.float32)).to(dev)
    so = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int32)).to(dev)
    g = gf.guide_field(lab, sg, so, eta=eta, cutoff=cutoff)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def _compare(label, seg, off, eta=3.0, cutoff=None):
    got = _gpu(label, seg, off, eta, cutoff)
    ref = oracle.guide_field(label, seg, off, eta=eta, cutoff=cutoff)
    assert got.shape == ref.shape
    # zero exactly where the oracle is zero (off the hole, beyond the cutoff)
    assert np.array_equal(got == 0, ref == 0)
    err = np.abs(got.astype(np.float64) - ref).max(initial=0.0)
    assert err <= TOL, err
    return got, ref


@pytest.mark.parametrize("B,H,W", [(1, 37, 53), (3, 64, 80), (2, 1, 1), (1, 33, 1031)])
def test_random_polylines(B, H, W):
    rng = np.random.default_rng(1000 + 7 * B + H + W)
    label = rng.choice([0, 1, 2], size=(B, H, W), p=[0.4, 0.5, 0.1]).astype(np.uint8)
    frames = []
    for b in range(B):
        n = 0 if b == 1 else int(rng.integers(1, 40))  # frame 1 has no spline
        a = rng.uniform(-5, max(H, W) + 5, size=(n, 2))
        c = a + rng.normal(0, 6, size=(n, 2))
        g = rng.normal(size=(n, 2))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        frames.append(np.concatenate([a, c, g], axis=1))
    seg, off = synthetic.pack_segments(frames)
    for eta, cutoff in [(3.0, None), (1.5, 2.0), (4.0, 0.0)]:
        _compare(label, seg, off, eta, cutoff)


def test_shared_vertices_and_degenerate_segments():
    # a polyline whose joints are equidistant from many pixels, repeated points
    # (zero-length segments) and a spline entirely outside the frame
    H, W = 40, 40
    label = np.ones((1, H, W), dtype=np.uint8)
    pts = np.array([[5, 5], [20, 5], [20, 5], [20, 30], [35, 30]], dtype=np.float64)
    rows = []
    for k in range(len(pts) - 1):
        d = pts[k + 1] - pts[k]
        n = np.linalg.norm(d)
        u = d / n if n > 0 else np.array([0.6, 0.8])
        rows.append([*pts[k], *pts[k + 1], *u])
    rows.append([-50, -50, -60, -40, 1.0, 0.0])
    seg, off = synthetic.pack_segments([np.array(rows)])
    got, ref = _compare(label, seg, off, 3.0, None)
    # the joint (20, 5) belongs to the first segment reaching it: direction (1, 0)
    assert got[0, 5, 20, 0] == 1.0 and got[0, 5, 20, 1] == 0.0


def test_full_frame_from_random_beziers():
    """1920 x 1080 with the silhouette holes and random Bezier splines of the
    plain full-HD workload, sampled every 2 px."""
    rng = np.random.default_rng(2)
    H, W = 1080, 1920
    label = synthetic.silhouette_bands(rng, H, W, n=6)
    seg = synthetic.spline_segments(rng, H, W, n_splines=6, spacing=2.0)
    seg, off = synthetic.pack_segments([seg])
    assert seg.shape[0] > 1000
    got, ref = _compare(label[None], seg, off)
    assert (np.abs(got) > 0).any()


def test_many_segments_per_tile_and_duplicates():
    """More segments than one staging batch near every tile, and exact
    duplicates (later copies with other directions): the first copy wins."""
    rng = np.random.default_rng(44)
    H, W = 70, 90
    label = (rng.uniform(size=(2, H, W)) < 0.6).astype(np.uint8)
    frames = []
    for b in range(2):
        n = 2600
        a = rng.uniform(0, [W, H], size=(n, 2))
        c = a + rng.normal(0, 2.0, size=(n, 2))
        g = rng.normal(size=(n, 2))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        seg = np.concatenate([a, c, g], axis=1)
        dup = seg[:300].copy()
        dup[:, 4:] = -dup[:, 4:]
        frames.append(np.concatenate([seg, dup]))
    seg, off = synthetic.pack_segments(frames)
    _compare(label, seg, off, 3.0, None)
    _compare(label, seg, off, 2.0, 1.5)
