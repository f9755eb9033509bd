"""Launch-shape autotuner: candidate set, cache, and (on the GPU) that the
tuned launch computes the same fill."""

import numpy as np
import pytest
import torch

import synthetic as syn


def test_candidates_are_valid_launch_shapes():
    import paper_1611_05319_amd as gf
    from paper_1611_05319_amd import autotune

    for shape, eps in (((1, 1080, 1920, 3), 3.0), ((1, 2160, 3840, 3), 5.0), ((4, 64, 80, 1), 2.0)):
        img = torch.zeros(shape)
        cands = autotune.candidates(img, gf.Params(eps=eps, mu=50.0, c=0.3, ghost=False))
        engines = {p.engine for p in cands}
        assert engines == {gf.ENGINE_TILED, gf.ENGINE_FRONT}
        keys = set()
        for p in cands:
            # method parameters are never tuned
            assert (p.eps, p.mu, p.c, p.ghost, p.tracking, p.max_shells) == (eps, 50.0, 0.3, False, True, 0)
            if p.engine == gf.ENGINE_TILED:
                tw, th, S, halo, lds, G = gf.tile_geometry(shape[1], shape[2], shape[3], img.dtype, p)
                assert halo <= min(tw, th)
            k = (p.engine, p.group, p.blocks_per_cu, p.tile_w, p.tile_h, p.pass_shells, p.tile_threads)
            assert k not in keys
            keys.add(k)


def test_cache_round_trip(tmp_path):
    from paper_1611_05319_amd import autotune

    path = str(tmp_path / "sub" / "tune.json")
    assert autotune._load_cache(path) == {}
    autotune._store_cache(path, "a", {"params": {"engine": 1}, "ms": 1.0})
    autotune._store_cache(path, "b", {"params": {"engine": 0}, "ms": 2.0})
    d = autotune._load_cache(path)
    assert d["a"]["params"]["engine"] == 1 and d["b"]["ms"] == 2.0
    (tmp_path / "bad.json").write_text("not json")
    assert autotune._load_cache(str(tmp_path / "bad.json")) == {}


@pytest.mark.gpu
def test_tuned_launch_fills_the_same(tmp_path):
    import paper_1611_05319_amd as gf
    from paper_1611_05319_amd import autotune

    w = syn.config1()
    dev = torch.device("cuda:0")
    img = torch.from_numpy(w.image).to(dev)
    lab = torch.from_numpy(w.label).to(dev)
    gd = torch.from_numpy(w.guide).to(dev)
    base = gf.Params(eps=w.eps, mu=w.mu)
    path = str(tmp_path / "tune.json")
    report = []
    p = autotune.tune(img, lab, gd, base, reps=2, path=path, report=report)
    assert len(report) >= 4
    again = []
    p2 = autotune.tune(img, lab, gd, base, reps=2, path=path, report=again)
    assert again == [] and p2 == p  # served from the cache
    ref = gf.fill_batched(img, lab, gd, base)
    got = gf.fill_batched(img, lab, gd, p)
    np.testing.assert_array_equal(got.shell.cpu().numpy(), ref.shell.cpu().numpy())
    a, b = got.out.cpu().numpy(), ref.out.cpu().numpy()
    assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-2)) <= 2e-6
