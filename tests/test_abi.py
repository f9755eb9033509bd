"""C ABI contract on the CPU: the library builds and loads, exports every
function the header declares, and rejects bad arguments synchronously
(argument checks run before any HIP call, so no device is needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "guidefill.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1611_05319_amd as gf
    from paper_1611_05319_amd import build

    if not os.path.exists(gf.library_path()):
        build.build()
    return gf.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(gf_[a-z_0-9]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("gf_fill", "gf_fill_batched", "gf_fill_backward", "gf_workspace_size",
              "gf_backward_workspace_size", "gf_status_string", "gf_last_error", "gf_version"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared_functions():
        assert hasattr(lib, n), n


def test_version_and_status_strings(lib):
    assert lib.gf_version() == 2
    assert lib.gf_status_string(0) == b"ok"
    assert lib.gf_status_string(-1) == b"invalid argument"
    assert lib.gf_status_string(-2) == b"HIP device error"
    assert lib.gf_status_string(-3) == b"unsupported request"


def test_workspace_size(lib):
    import paper_1611_05319_amd as gf

    p = gf.Params(engine=gf.ENGINE_FRONT).c_struct()
    n1 = lib.gf_workspace_size(1, 1080, 1920, 3, 0, ctypes.byref(p))
    n2 = lib.gf_workspace_size(2, 1080, 1920, 3, 0, ctypes.byref(p))
    assert n1 >= 2 * 1080 * 1920 * 4 and n2 > n1
    assert n1 % 256 == 0
    t = gf.Params().c_struct()  # tiled engine: per-tile words only
    m1 = lib.gf_workspace_size(1, 1080, 1920, 3, 0, ctypes.byref(t))
    m2 = lib.gf_workspace_size(4, 1080, 1920, 3, 0, ctypes.byref(t))
    assert 0 < m1 < n1 and m2 > m1
    assert lib.gf_workspace_size(0, 10, 10, 3, 0, ctypes.byref(p)) == 0
    assert lib.gf_backward_workspace_size(1, 10, 10, 3, 0, ctypes.byref(p)) >= 256


def _call(lib, params, B=1, H=8, W=8, C=3, dt=0, ptr=1 << 20, ws_bytes=1 << 20, ws=1 << 20,
          kcap=0, order=None, offs=None):
    P = ctypes.c_void_p
    fake = P(ptr)
    return lib.gf_fill_batched(fake, fake, B, H, W, C, dt, fake, fake, ctypes.byref(params),
                               fake, fake, order, offs, None, kcap, P(ws), ws_bytes, None)


@pytest.mark.parametrize("field,value", [
    ("eps", 0.0), ("eps", 0.5), ("eps", 9.5), ("eps", float("nan")), ("mu", 0.0),
    ("mu", -1.0), ("mu", float("inf")), ("c", float("nan")), ("max_shells", -1),
    ("group", 2), ("blocks_per_cu", 9), ("blocks_per_cu", -1), ("engine", 2), ("engine", -1),
    ("pass_shells", 33), ("pass_shells", -1), ("tile_w", 300), ("tile_h", -2),
    ("tile_threads", 128), ("tile_threads", 640), ("tile_threads", -256)])
def test_bad_parameters_are_rejected(lib, field, value):
    import paper_1611_05319_amd as gf

    p = gf.Params()
    setattr(p, field, value)
    assert _call(lib, p.c_struct()) == -1


def test_data_term_needs_one_frame(lib):
    import paper_1611_05319_amd as gf

    assert _call(lib, gf.Params(c2=0.0).c_struct(), B=2) == -3
    assert _call(lib, gf.Params(c2=float("nan")).c_struct()) == -1


def test_tile_threads_only_with_the_tiled_engine(lib):
    import paper_1611_05319_amd as gf

    assert _call(lib, gf.Params(engine=gf.ENGINE_FRONT, tile_threads=256).c_struct()) == -1
    assert _call(lib, gf.Params(engine=gf.ENGINE_FRONT, group=4).c_struct()) == -1
    # 4 lanes hold at most 32 offsets and need floor(eps) < 4
    assert _call(lib, gf.Params(group=4, eps=3.6).c_struct()) == -3


@pytest.mark.parametrize("shape", [(0, 8, 8, 3), (1, 0, 8, 3), (1, 8, 0, 3), (1, 8, 8, 0),
                                   (1, 8, 8, 5)])
def test_bad_shapes_are_rejected(lib, shape):
    import paper_1611_05319_amd as gf

    B, H, W, C = shape
    assert _call(lib, gf.Params().c_struct(), B=B, H=H, W=W, C=C) == -1


def test_tile_halo_must_fit_the_neighbour_tiles(lib):
    import paper_1611_05319_amd as gf

    # halo pass_shells * ceil(eps) = 12 > tile 8: the tile tracking would be inexact
    p = gf.Params(tile_w=8, tile_h=8, pass_shells=4).c_struct()
    assert _call(lib, p) == -1
    out = (ctypes.c_int32 * 6)()
    assert lib.gf_tile_geometry(64, 64, 3, 0, ctypes.byref(p), out) == -1
    q = gf.Params().c_struct()
    assert lib.gf_tile_geometry(1080, 1920, 3, 0, ctypes.byref(q), out) == 0
    tw, th, S, halo, lds, G = list(out)
    assert halo == S * 3 and halo <= tw and halo <= th and G in (8, 16, 32, 64)
    # 8 lanes hold at most 32 ball offsets: eps = 5 (80 offsets) needs a wider group
    for engine in (gf.ENGINE_TILED, gf.ENGINE_FRONT):
        f = gf.Params(engine=engine, group=8, eps=5.0).c_struct()
        assert _call(lib, f) == -3
    q5 = gf.Params(eps=5.0, mu=100.0).c_struct()
    assert lib.gf_tile_geometry(2160, 3840, 3, 0, ctypes.byref(q5), out) == 0
    assert out[3] == out[2] * 5 and out[3] <= out[0]


def test_order_needs_the_front_engine(lib):
    import paper_1611_05319_amd as gf

    p = gf.Params(engine=gf.ENGINE_TILED).c_struct()
    assert _call(lib, p, order=ctypes.c_void_p(1 << 20), offs=ctypes.c_void_p(1 << 21),
                 kcap=4) == -3


def test_bad_pointers_and_workspace_are_rejected(lib):
    import paper_1611_05319_amd as gf

    p = gf.Params().c_struct()
    assert _call(lib, p, ptr=0) == -1               # null device pointers
    assert _call(lib, p, ws_bytes=16) == -1          # workspace too small
    assert _call(lib, p, ws=(1 << 20) + 8) == -1     # misaligned workspace
    assert _call(lib, p, dt=7) == -1                 # unknown dtype
    # order_out without shell_offsets (and the reverse)
    assert _call(lib, p, order=ctypes.c_void_p(1 << 20), kcap=4) == -1
    assert _call(lib, p, offs=ctypes.c_void_p(1 << 20), kcap=4) == -1
    # too many pixels for int32 list entries
    big = gf.Params().c_struct()
    assert _call(lib, big, B=1 << 12, H=1 << 10, W=1 << 10, ws_bytes=1 << 62) == -3


def test_backward_rejects_bad_arguments(lib):
    import paper_1611_05319_amd as gf

    P = ctypes.c_void_p
    fake = P(1 << 20)
    p = gf.Params().c_struct()
    nbytes = lib.gf_backward_workspace_size(1, 8, 8, 3, 0, ctypes.byref(p))
    # control block, shell counts, H * W + 2 shell offsets, B * H * W order entries
    assert nbytes >= 4096 + 2 * 2048 * 4 + (64 + 2) * 4 + 64 * 4 and nbytes % 256 == 0

    def call(shell=fake, K=2, ws_bytes=nbytes, ws=fake, grad=fake, params=p):
        return lib.gf_fill_backward(grad, fake, 1, 8, 8, 3, 0, None, fake, shell, K,
                                    ctypes.byref(params), fake, fake, ws, ws_bytes, None)

    assert call(shell=None) == -1              # no shell map
    assert call(grad=None) == -1               # no grad_out
    assert call(K=-2) == -1                    # K below -1
    assert call(K=65) == -1                    # more shells than pixels in a frame
    assert call(ws_bytes=nbytes - 256) == -1   # workspace too small
    assert call(ws=P((1 << 20) + 8)) == -1     # misaligned workspace
    assert call(params=gf.Params(eps=0.5).c_struct()) == -1


def test_python_binding_fails_loudly_without_device():
    import torch

    import paper_1611_05319_amd as gf

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    img = torch.zeros(4, 4, 3)
    lab = torch.zeros(4, 4, dtype=torch.uint8)
    g = torch.zeros(4, 4, 2)
    with pytest.raises(ValueError):
        gf.fill(img, lab, g)


def test_noalloc_rejects_requests_beyond_the_scratch(lib):
    """The no-allocation entry point checks the workspace it would need against
    its static scratch before any HIP call."""
    import paper_1611_05319_amd as gf

    p = gf.Params(engine=gf.ENGINE_FRONT).c_struct()
    fake = ctypes.c_void_p(1 << 20)
    # two 1920 x 1080 frames need two front lists of 2 x 8.3 MB: beyond 16 MiB
    assert lib.gf_workspace_size(2, 1080, 1920, 3, 0, ctypes.byref(p)) > gf.SCRATCH_BYTES
    rc = lib.gf_fill_batched_noalloc(fake, fake, 2, 1080, 1920, 3, 0, fake, fake, ctypes.byref(p),
                                     fake, fake, None, None, None, 0, None)
    assert rc == -1
    assert b"scratch" in lib.gf_last_error()
    bad = gf.Params(eps=0.5).c_struct()
    assert lib.gf_fill_batched_noalloc(fake, fake, 1, 8, 8, 3, 0, fake, fake, ctypes.byref(bad),
                                       fake, fake, None, None, None, 0, None) == -1


def test_guide_field_rejects_bad_arguments(lib):
    fake = ctypes.c_void_p(1 << 20)
    for B, H, W, eta, cutoff in [(0, 8, 8, 3.0, 9.0), (1, 0, 8, 3.0, 9.0), (1, 8, 8, 0.0, 9.0),
                                 (1, 8, 8, 3.0, -1.0), (1, 8, 8, float("nan"), 9.0),
                                 (1, 8, 8, 3.0, float("inf"))]:
        assert lib.gf_guide_field(B, H, W, fake, fake, fake, eta, cutoff, fake, None) == -1
    assert lib.gf_guide_field(1, 8, 8, None, fake, fake, 3.0, 9.0, fake, None) == -1
    assert lib.gf_guide_field(1, 8, 8, fake, fake, None, 3.0, 9.0, fake, None) == -1
    assert lib.gf_guide_field(1, 8, 8, fake, fake, fake, 3.0, 9.0, None, None) == -1


def test_coherence_rejects_bad_arguments(lib):
    import paper_1611_05319_amd as gf

    fake = ctypes.c_void_p(1 << 20)
    p = gf.Params(ghost=False).c_struct()
    n = lib.gf_coherence_workspace_size(2, 40, 50, 3, 0, ctypes.byref(p))
    # its one-shell fills run one shell per pass
    p1 = gf.Params(ghost=False, max_shells=1, pass_shells=1).c_struct()
    nf = lib.gf_workspace_size(2, 40, 50, 3, 0, ctypes.byref(p1))
    assert n % 256 == 0 and n >= nf + 2 * 40 * 50 * (1 + 8 + 4)
    assert lib.gf_coherence_workspace_size(0, 40, 50, 3, 0, ctypes.byref(p)) == 0

    def call(sigma=2.0, rho=4.0, lam=1e-5, params=p, ws=n, shell=fake):
        return lib.gf_fill_coherence(fake, fake, 2, 40, 50, 3, 0, fake, ctypes.byref(params), sigma,
                                     rho, lam, shell, fake, None, fake, ws, None)

    assert call(sigma=0.0) == -1
    assert call(rho=-1.0) == -1
    assert call(lam=0.0) == -1
    assert call(lam=float("inf")) == -1
    assert call(sigma=9.0) == -3
    assert call(rho=17.0) == -3
    assert call(ws=n - 256) == -1
    assert call(shell=None) == -1
    p2 = gf.Params(ghost=False, c2=0.1).c_struct()
    assert call(params=p2) == -3
