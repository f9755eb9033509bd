"""gf_fill_batched_noalloc (the entry point for callers that cannot allocate:
it runs on the library's static per-device scratch) against gf_fill_batched
with a caller-allocated workspace, through the C ABI: two calls in a row, the
second on a smaller input, must give the same shell maps (bit-exact), colours
(bit-exact: the same kernels run) and statistics."""

import ctypes

import numpy as np
import pytest

import synthetic as syn
from gpu_helpers import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1611_05319_amd as gf

    return gf.load()


def _buffers(w, dtype):
    import torch

    dev = torch.device("cuda:0")
    img = torch.from_numpy(w.image).to(dev).to(dtype).contiguous()
    lab = torch.from_numpy(w.label).to(dev)
    gd = torch.from_numpy(w.guide).to(dev)
    B, H, W, C = img.shape
    outs = []
    for _ in range(2):  # one set for each entry point
        outs.append((torch.empty_like(img), torch.empty((B, H, W), dtype=torch.int32, device=dev),
                     torch.empty(8 + 4 * B, dtype=torch.int32, device=dev)))
    return img, lab, gd, outs


def _run_both(lib, w, params, dtype):
    """Both entry points on the same inputs; returns their (out, shell, stats)."""
    import torch

    import paper_1611_05319_amd as gf

    img, lab, gd, ((o1, s1, t1), (o2, s2, t2)) = _buffers(w, dtype)
    B, H, W, C = img.shape
    dt = 1 if dtype == torch.float16 else 0
    cp = params.c_struct()
    nbytes = lib.gf_workspace_size(B, H, W, C, dt, ctypes.byref(cp))
    assert 0 < nbytes <= gf.SCRATCH_BYTES
    ws = torch.zeros(nbytes, dtype=torch.uint8, device=img.device)
    torch.cuda.synchronize()
    P = ctypes.c_void_p
    stream = P(torch.cuda.current_stream().cuda_stream)
    rc = lib.gf_fill_batched(P(img.data_ptr()), P(o1.data_ptr()), B, H, W, C, dt, P(lab.data_ptr()),
                             P(gd.data_ptr()), ctypes.byref(cp), P(s1.data_ptr()), P(t1.data_ptr()),
                             None, None, None, 0, P(ws.data_ptr()), ws.numel(), stream)
    assert rc == 0, lib.gf_last_error()
    rc = lib.gf_fill_batched_noalloc(P(img.data_ptr()), P(o2.data_ptr()), B, H, W, C, dt,
                                     P(lab.data_ptr()), P(gd.data_ptr()), ctypes.byref(cp),
                                     P(s2.data_ptr()), P(t2.data_ptr()), None, None, None, 0, stream)
    assert rc == 0, lib.gf_last_error()
    torch.cuda.synchronize()
    return [(o.float().cpu().numpy(), s.cpu().numpy(), gf.stats_fields(t)) for o, s, t in
            ((o1, s1, t1), (o2, s2, t2))]


def _assert_same(a, b):
    (u1, s1, st1), (u2, s2, st2) = a, b
    np.testing.assert_array_equal(s2, s1)
    np.testing.assert_array_equal(u2, u1)
    for key in ("K", "filled", "hole", "label_errors", "frame_K", "frame_filled", "frame_hole"):
        assert st2[key] == st1[key], key
    assert not st1["sync_timeout"] and not st2["sync_timeout"]
    assert st1["filled"] > 0


@pytest.mark.parametrize("engine", [0, 1])
def test_noalloc_matches_the_workspace_call_twice(lib, engine):
    import torch

    import paper_1611_05319_amd as gf

    big = syn.config2()     # 1920 x 1080, binary32
    small = syn.config1()   # 256 x 256, binary32
    for name, w in (("1920x1080", big), ("256x256", small)):
        banner(f"noalloc engine={engine} {name}")
        p = gf.Params(eps=w.eps, mu=w.mu, engine=engine)
        a, b = _run_both(lib, w, p, torch.float32)
        _assert_same(a, b)


def test_noalloc_batched_fp16_then_single_frame(lib):
    import torch

    import paper_1611_05319_amd as gf

    rng = np.random.default_rng(31)
    frames = [syn.random_tiny(rng, 96, 128, C=3, p_hole=p, p_bystander=0.05) for p in (0.1, 0.4, 0.7)]

    class W:
        pass

    w = W()
    w.image = np.stack([f[0] for f in frames])
    w.label = np.stack([f[1] for f in frames])
    w.guide = np.stack([f[2] for f in frames])
    w1 = W()
    w1.image, w1.label, w1.guide = w.image[1:2, :40, :50], w.label[1:2, :40, :50], w.guide[1:2, :40, :50]
    w1.image, w1.label, w1.guide = (np.ascontiguousarray(x) for x in (w1.image, w1.label, w1.guide))
    for name, ww in (("3 x 96x128 fp16", w), ("1 x 40x50 fp16", w1)):
        banner(f"noalloc {name}")
        a, b = _run_both(lib, ww, gf.Params(), torch.float16)
        _assert_same(a, b)


def test_noalloc_rejects_requests_beyond_the_scratch(lib):
    import paper_1611_05319_amd as gf

    banner("noalloc: oversize request")
    # two 1080p frames on the global-front engine need two 2 x 8.3 MB front lists
    p = gf.Params(engine=gf.ENGINE_FRONT).c_struct()
    fake = ctypes.c_void_p(1 << 20)
    rc = lib.gf_fill_batched_noalloc(fake, fake, 2, 1080, 1920, 3, 0, fake, fake, ctypes.byref(p),
                                     fake, fake, None, None, None, 0, None)
    assert rc == -1
    assert b"scratch" in lib.gf_last_error()
