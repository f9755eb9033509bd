"""HIP path against the FP64 oracle, element by element, through the C ABI.

Shell maps must be bit-exact; binary32 colours within 1e-5 relative
(max(|ref|, 1e-2) floor); tracked and untracked forms, batched and single
frames, in place and out of place must agree with each other exactly."""

import math

import numpy as np
import pytest

import oracle
import synthetic as syn
from gpu_helpers import assert_colour_parity, banner, f16_one_step, f16_ulps, gpu_fill

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1611_05319_amd as gf

    gf.load()


# launch variants: the tiled engine (default 768-thread, 1024- and 256-thread
# workgroups; the 1024-thread form stages its windows in two round trips, the
# others in one) and the global-front engine
LAUNCH = {"tiled": {}, "tiled1024": {"tile_threads": 1024}, "tiled256": {"tile_threads": 256},
          "front": {"engine": 1}}
ENGINES = list(LAUNCH)


def _check(img, lab, g, eps=3.0, mu=50.0, c=-1.0, ghost=True, tracking=True, ref=None, **kw):
    if ref is None:
        ref = oracle.fill(img, lab, g, eps=eps, mu=mu, c=c, ghost=ghost)
    u, s, st, _ = gpu_fill(img, lab, g, eps=eps, mu=mu, c=c, ghost=ghost, tracking=tracking, **kw)
    np.testing.assert_array_equal(s, ref.shell)
    worst = assert_colour_parity(u, ref.u, ref.shell)
    # pixels that are not filled keep their input colour exactly
    keep = ref.shell < 0
    np.testing.assert_array_equal(u[keep], img[keep].astype(np.float64))
    assert st["K"] == ref.K and st["filled"] == ref.n_filled and st["hole"] == ref.stats[0, 4]
    return ref, u, s, st, worst


def test_config1_tracked_and_untracked():
    w = syn.config1()
    for engine in ENGINES:
        for tracking in (True, False):
            for ghost in (True, False):
                banner(f"c1 engine={engine} tracking={tracking} ghost={ghost}")
                _check(w.image[0], w.label[0], w.guide[0], ghost=ghost, tracking=tracking,
                       **LAUNCH[engine])


CASES = [
    # (H, W, C, eps, mu, c, ghost, p_hole, p_bys)
    (1, 1, 3, 3.0, 50.0, -1.0, True, 0.5, 0.0),
    (1, 23, 3, 3.0, 50.0, -1.0, True, 0.4, 0.1),
    (29, 1, 1, 3.0, 50.0, -1.0, False, 0.4, 0.1),
    (5, 7, 3, 3.0, 50.0, -1.0, True, 0.5, 0.1),
    (33, 65, 3, 3.0, 50.0, -1.0, True, 0.35, 0.1),
    (64, 64, 4, 2.0, 10.0, -1.0, True, 0.4, 0.05),
    (97, 130, 3, 3.6, 20.0, -1.0, True, 0.3, 0.1),
    (71, 90, 2, 5.0, 100.0, -1.0, True, 0.4, 0.1),
    (71, 90, 3, 5.0, 100.0, -1.0, False, 0.4, 0.1),
    (80, 77, 3, 3.0, 50.0, 0.05, True, 0.35, 0.1),
    (80, 77, 1, 3.0, 5.0, 0.3, False, 0.35, 0.1),
    (128, 256, 3, 3.0, 50.0, -1.0, True, 0.6, 0.0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}-e{c[3]}-c{c[5]}-g{int(c[6])}" for c in CASES])
@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("tracking", [True, False])
def test_random_problems(case, tracking, engine):
    H, W, C, eps, mu, c, ghost, ph, pb = case
    banner(f"random {case} tracking={tracking} engine={engine}")
    rng = np.random.default_rng(hash(case) % (1 << 32))
    img, lab, g = syn.random_tiny(rng, H, W, C=C, p_hole=ph, p_bystander=pb,
                                  blob=min(H, W) > 4)
    ref = oracle.fill(img, lab, g, eps=eps, mu=mu, c=c, ghost=ghost)
    if c >= 0:
        assert ref.n_ties == 0, "confidence within the tie band of the threshold"
    _check(img, lab, g, eps=eps, mu=mu, c=c, ghost=ghost, tracking=tracking, ref=ref,
           **LAUNCH[engine])


def test_lattice_line_angles():
    # angles that put ghost points exactly on lattice lines (30, 45, 90 degrees)
    rng = np.random.default_rng(3)
    H, W = 60, 70
    img, lab, g = syn.random_tiny(rng, H, W, C=3, p_hole=0.45, p_bystander=0.05)
    angles = np.deg2rad(np.array([0.0, 30.0, 45.0, 60.0, 90.0, 150.0, 210.0, 270.0]))
    pick = rng.integers(0, len(angles), size=(H, W))
    g = np.stack([np.cos(angles[pick]), np.sin(angles[pick])], -1).astype(np.float32)
    g = np.where((lab == 1)[..., None], g, np.float32(0))
    ref = oracle.fill(img, lab, g)
    for engine in ENGINES:
        for tracking in (True, False):
            banner(f"lattice-line angles tracking={tracking} engine={engine}")
            _check(img, lab, g, tracking=tracking, **LAUNCH[engine], ref=ref)


@pytest.mark.parametrize("engine", ENGINES)
def test_edge_cases(engine):
    rng = np.random.default_rng(8)
    img = rng.uniform(0, 1, size=(40, 50, 3)).astype(np.float32)
    g = np.zeros((40, 50, 2), np.float32)
    g[..., 0] = 1.0
    # no hole at all
    banner("edge: no hole")
    lab = np.zeros((40, 50), np.uint8)
    ref, u, s, st, _ = _check(img, lab, g, **LAUNCH[engine])
    assert st["K"] == 0 and st["hole"] == 0
    # everything is hole: nothing readable, nothing filled
    banner("edge: all hole")
    lab = np.ones((40, 50), np.uint8)
    ref, u, s, st, _ = _check(img, lab, g, **LAUNCH[engine])
    assert (s == -3).all() and st["filled"] == 0
    # hole surrounded by bystanders (stall), and a hole on the image border
    banner("edge: stall")
    lab = np.zeros((40, 50), np.uint8)
    lab[10:30, 10:30] = 2
    lab[15:25, 15:25] = 1
    lab[0:3, 40:50] = 1
    ref, u, s, st, _ = _check(img, lab, g, **LAUNCH[engine])
    assert (s[15:25, 15:25] == -3).all() and st["unfilled"] == 100
    # label values outside {0, 1, 2} are counted and act as bystanders
    banner("edge: bad labels")
    lab = np.zeros((40, 50), np.uint8)
    lab[5:12, 5:30] = 1
    lab[20, 20] = 7
    ref_lab = lab.copy()
    ref_lab[20, 20] = 2
    ref = oracle.fill(img, ref_lab, g)
    u, s, st, _ = gpu_fill(img, lab, g, **LAUNCH[engine])
    np.testing.assert_array_equal(s, ref.shell)
    assert st["label_errors"] == 1


def test_constant_image_is_exact():
    banner("constant image")
    rng = np.random.default_rng(4)
    img, lab, g = syn.random_tiny(rng, 90, 110, C=3, p_hole=0.4, p_bystander=0.1)
    img[:] = np.array([0.25, 0.7, 1.0 / 3.0], np.float32)
    u, s, _, _ = gpu_fill(img, lab, g)
    filled = s >= 0
    assert filled.sum() > 100
    np.testing.assert_array_equal(u[filled], np.broadcast_to(img[0, 0].astype(np.float64),
                                                            u[filled].shape))


FORMS = [
    {"engine": 1}, {"engine": 1, "tracking": False}, {"tracking": False}, {"inplace": True},
    {"engine": 1, "inplace": True}, {"group": 8}, {"group": 16}, {"group": 32}, {"group": 64},
    {"engine": 1, "group": 16}, {"blocks_per_cu": 1}, {"blocks_per_cu": 4},
    {"tile_w": 12, "tile_h": 12, "pass_shells": 1}, {"tile_w": 16, "tile_h": 24, "pass_shells": 2},
    {"tile_w": 24, "tile_h": 24, "pass_shells": 6},
    {"tile_w": 64, "tile_h": 16, "pass_shells": 5}, {"tile_w": 20, "tile_h": 36, "pass_shells": 3},
    {"tile_w": 24, "tile_h": 24, "pass_shells": 7, "tracking": False},
    {"tile_w": 48, "tile_h": 48, "pass_shells": 2}, {"tile_w": 20, "tile_h": 20, "pass_shells": 6},
    {"tile_w": 27, "tile_h": 27, "pass_shells": 7},
    {"tile_threads": 256}, {"tile_threads": 512}, {"tile_threads": 512, "pass_shells": 2},
    {"group": 4}, {"group": 4, "tile_threads": 512}, {"group": 4, "tracking": False},
    {"tile_threads": 768}, {"tile_threads": 768, "group": 16, "pass_shells": 3},
    {"tile_threads": 1024}, {"tile_threads": 1024, "group": 16, "pass_shells": 3},
    {"tile_threads": 256, "tile_w": 16, "tile_h": 16, "pass_shells": 4},
    {"tile_threads": 256, "tile_w": 24, "tile_h": 12, "pass_shells": 2, "tracking": False},
    {"tile_threads": 256, "tile_w": 16, "tile_h": 16, "group": 16},
    {"tile_threads": 256, "tile_w": 16, "tile_h": 16, "blocks_per_cu": 2}, {},
]


def test_forms_agree_exactly():
    banner("forms: engines, tracking, in place, groups, tiles, repeat")
    w = syn.config1(seed=11, H=200, W=240)
    img, lab, g = w.image[0], w.label[0], w.guide[0]
    ref = oracle.fill(img, lab, g)
    u0, s0, st0, _ = gpu_fill(img, lab, g)
    np.testing.assert_array_equal(s0, ref.shell)
    import paper_1611_05319_amd as gf

    for kw in FORMS:
        banner(f"form {kw}")
        u1, s1, st1, _ = gpu_fill(img, lab, g, **kw)
        np.testing.assert_array_equal(s1, s0)
        G = kw.get("group") or 8
        if G != 8:  # another reduction tree: the last FP64 bits may differ
            assert np.abs(u1 - u0).max() <= 2.0 ** -23
        else:
            np.testing.assert_array_equal(u1, u0)
        assert st1["K"] == st0["K"] and st1["filled"] == st0["filled"]
    # batched frames give the per-frame results
    rng = np.random.default_rng(12)
    frames = [syn.random_tiny(rng, 64, 80, C=3, p_hole=p, p_bystander=0.05) for p in (0.1, 0.3, 0.6)]
    bi = np.stack([f[0] for f in frames])
    bl = np.stack([f[1] for f in frames])
    bg = np.stack([f[2] for f in frames])
    for engine in ENGINES:
        ub, sb, stb, _ = gpu_fill(bi, bl, bg, **LAUNCH[engine])
        for i, (fi, fl, fg) in enumerate(frames):
            ui, si, sti, _ = gpu_fill(fi, fl, fg, **LAUNCH[engine])
            np.testing.assert_array_equal(sb[i], si)
            np.testing.assert_array_equal(ub[i], ui)
            assert stb["frame_K"][i] == sti["K"] and stb["frame_filled"][i] == sti["filled"]
            assert stb["frame_hole"][i] == sti["hole"]


# windows that do not fit: more than 8192 window pixels (uint16 local lists),
# or more LDS than one workgroup may use (32 bytes per window pixel)
OVERSIZE = [{"tile_w": 100, "tile_h": 120, "pass_shells": 2}, {"tile_w": 40, "tile_h": 40, "pass_shells": 8},
            {"tile_w": 24, "tile_h": 24, "pass_shells": 8}]


@pytest.mark.parametrize("kw", OVERSIZE)
def test_oversize_windows_are_rejected(kw):
    import paper_1611_05319_amd as gf

    banner(f"oversize window {kw}")
    with pytest.raises(RuntimeError, match="invalid argument"):
        gf.tile_geometry(200, 240, 3, params=gf.Params(**kw))
    w = syn.config1(seed=11, H=200, W=240)
    with pytest.raises(RuntimeError, match="invalid argument"):
        gpu_fill(w.image[0], w.label[0], w.guide[0], **kw)


def test_single_frame_entry_point():
    """gf_fill (one frame) called directly through the C ABI."""
    import ctypes

    import torch

    import paper_1611_05319_amd as gf

    lib = gf.load()
    w = syn.config1(seed=13, H=180, W=220)
    img, lab, g = w.image[0], w.label[0], w.guide[0]
    ref = oracle.fill(img, lab, g)
    dev = torch.device("cuda:0")
    for engine in (0, 1):
        banner(f"gf_fill engine={engine}")
        ti, tl, tg = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (img, lab, g))
        out = torch.empty_like(ti)
        shell = torch.empty(lab.shape, dtype=torch.int32, device=dev)
        stats = torch.empty(12, dtype=torch.int32, device=dev)
        cp = gf.Params(engine=engine).c_struct()
        nbytes = lib.gf_workspace_size(1, *lab.shape, 3, 0, ctypes.byref(cp))
        ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        P = ctypes.c_void_p
        rc = lib.gf_fill(P(ti.data_ptr()), P(out.data_ptr()), lab.shape[0], lab.shape[1], 3, 0,
                         P(tl.data_ptr()), P(tg.data_ptr()), ctypes.byref(cp), P(shell.data_ptr()),
                         P(stats.data_ptr()), P(ws.data_ptr()), nbytes,
                         P(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, lib.gf_last_error()
        torch.cuda.synchronize()
        s = shell.cpu().numpy()
        np.testing.assert_array_equal(s, ref.shell)
        assert_colour_parity(out.cpu().numpy().astype(np.float64), ref.u, ref.shell)
        st = gf.stats_fields(stats)
        assert st["K"] == ref.K and st["filled"] == ref.n_filled and not st["sync_timeout"]


def test_front_sizes_match_active_boundary():
    # the tracked front of shell k is exactly the active boundary of D^(k)
    banner("front sizes")
    rng = np.random.default_rng(6)
    img, lab, g = syn.random_tiny(rng, 120, 150, C=3, p_hole=0.5, p_bystander=0.08)
    for ghost in (True, False):
        ref = oracle.fill(img, lab, g, ghost=ghost)
        K = ref.K
        for tracking in (True, False):
            # the tiled engine recounts only the tiles it visits: exact when no
            # pixel waits, which the lattice ball guarantees
            for engine in (["front", "tiled", "tiled256"] if not ghost else ["front"]):
                u, s, st, r = gpu_fill(img, lab, g, ghost=ghost, tracking=tracking,
                                       **LAUNCH[engine], record_fronts=True)
                hist = r.front_hist.cpu().numpy()
                np.testing.assert_array_equal(hist[:K], ref.front_hist[0, :K])
                assert st["max_front"] == ref.max_front


@pytest.mark.parametrize("engine", ENGINES)
def test_max_shells_resume(engine):
    banner("max_shells resume")
    rng = np.random.default_rng(9)
    img, lab, g = syn.random_tiny(rng, 100, 120, C=3, p_hole=0.5, p_bystander=0.05)
    u_full, s_full, st_full, _ = gpu_fill(img, lab, g, **LAUNCH[engine])
    assert st_full["K"] >= 4
    m = 3 if engine == "front" else 5  # 5 is not a multiple of the tiled engine's shells per pass
    u1, s1, st1, _ = gpu_fill(img, lab, g, max_shells=m, **LAUNCH[engine])
    assert st1["K"] == m
    lab2 = lab.copy()
    lab2[s1 >= 0] = 0
    u2, s2, _, _ = gpu_fill(u1.astype(np.float32), lab2, g, **LAUNCH[engine])
    s = np.where(s2 >= 0, s2 + m, s1)
    s = np.where((lab == 1) & (s1 >= 0), s1, s)
    np.testing.assert_array_equal(s, s_full)
    np.testing.assert_array_equal(u2, u_full)


@pytest.mark.parametrize("engine", ENGINES)
def test_fp16_storage(engine):
    import torch

    banner("fp16 storage")
    rng = np.random.default_rng(10)
    img, lab, g = syn.random_tiny(rng, 150, 170, C=3, p_hole=0.4, p_bystander=0.05)
    img16 = img.astype(np.float16)
    ref = oracle.fill(img16.astype(np.float64), lab, g, storage="f16")
    u, s, st, _ = gpu_fill(img16.astype(np.float32), lab, g, dtype=torch.float16, **LAUNCH[engine])
    np.testing.assert_array_equal(s, ref.shell)
    filled = s >= 0
    ulps = f16_ulps(u[filled], ref.u[filled])
    assert ulps.max() <= 1.0, f"{ulps.max()} binary16 spacings"
    assert (ulps > 0).mean() < 1e-3


def test_config2_full_size():
    w = syn.config2()
    img, lab, g = w.image[0], w.label[0], w.guide[0]
    ref = oracle.fill(img, lab, g)
    for engine in ENGINES:
        for tracking in (True, False):
            banner(f"c2 1920x1080 tracking={tracking} engine={engine}")
            ref, u, s, st, worst = _check(img, lab, g, tracking=tracking, **LAUNCH[engine], ref=ref)
            banner(f"c2 K={st['K']} N={st['filled']} worst rel err {worst:.2e}")


@pytest.mark.parametrize("config", ["c1", "c2"])
def test_smart_order_full_size(config):
    """Smart order (eqn:ready, c = 0.05) on the 256x256 and 1920x1080 frames:
    the oracle reports no confidence within its tie band of the threshold, so
    the shell maps must agree bit for bit."""
    w = syn.config1() if config == "c1" else syn.config2()
    img, lab, g = w.image[0], w.label[0], w.guide[0]
    ref = oracle.fill(img, lab, g, eps=w.eps, mu=w.mu, c=0.05)
    assert ref.n_ties == 0, "confidence within the tie band of the threshold"
    for engine in ENGINES:
        for tracking in (True, False):
            banner(f"smart order {config} c=0.05 engine={engine} tracking={tracking}")
            ref, u, s, st, worst = _check(img, lab, g, eps=w.eps, mu=w.mu, c=0.05, tracking=tracking,
                                          ref=ref, **LAUNCH[engine])
            banner(f"smart order {config}: K={st['K']} worst rel err {worst:.2e}")


def _guided_half(w):
    """The frame with its guide kept on the left half of the hole only."""
    img, lab, g = w.image[0], w.label[0], w.guide[0].copy()
    g[:, g.shape[1] // 2:] = 0.0
    return img, lab, g


@pytest.mark.parametrize("c", [-1.0, 0.05])
@pytest.mark.parametrize("c2", [0.0, 0.5])
@pytest.mark.parametrize("engine", ENGINES)
def test_data_term_ready2(engine, c2, c):
    """eqn:ready2 (data term |g| > c2 until it leaves nothing ready, then
    eqn:ready) on random problems with many zero guides, and on the
    1920x1080 frame with the guide removed from its right half."""
    rng = np.random.default_rng(int(c2 * 10) + (3 if c > 0 else 0))
    for i in range(3):
        img, lab, g = syn.random_tiny(rng, 70 + 9 * i, 90 - 7 * i, C=3, p_hole=0.45,
                                      p_bystander=0.05, zero_guide_frac=0.4)
        ref = oracle.fill(img, lab, g, c=c, c2=c2)
        if c >= 0:
            assert ref.n_ties == 0
        for tracking in (True, False):
            banner(f"ready2 random {i} c={c} c2={c2} engine={engine} tracking={tracking}")
            _check(img, lab, g, c=c, c2=c2, tracking=tracking, ref=ref, **LAUNCH[engine])
    w = syn.config2()
    img, lab, g = _guided_half(w)
    ref = oracle.fill(img, lab, g, eps=w.eps, mu=w.mu, c=c, c2=c2)
    assert ref.n_ties == 0
    banner(f"ready2 1920x1080 half guided c={c} c2={c2} engine={engine}")
    ref, u, s, st, worst = _check(img, lab, g, eps=w.eps, mu=w.mu, c=c, c2=c2, ref=ref,
                                  **LAUNCH[engine])
    plain = oracle.fill(img, lab, g, eps=w.eps, mu=w.mu, c=c)
    banner(f"ready2 1920x1080: K={st['K']} (without the data term {plain.K}), worst {worst:.2e}")


def test_config3_full_size():
    w = syn.config3()
    ref = oracle.fill(w.image[0], w.label[0], w.guide[0], eps=5.0, mu=100.0)
    # the launch forms, and the one the autotuner picks for the benchmark's
    # deep-front leg (global front, 16 lanes per pixel)
    forms = dict(LAUNCH, front16={"engine": 1, "group": 16})
    for engine, kw in forms.items():
        banner(f"c3 3840x2160 eps=5 mu=100 engine={engine}")
        ref, u, s, st, worst = _check(w.image[0], w.label[0], w.guide[0], eps=5.0, mu=100.0,
                                      ref=ref, **kw)
        banner(f"c3 K={st['K']} N={st['filled']} worst rel err {worst:.2e}")
        assert st["K"] > 50


@pytest.fixture(scope="module")
def config4_reference():
    """The 64-frame binary16 batch and the oracle's fill of every frame
    (binary16 rounding of inputs and of each fill)."""
    banner("c4 64 x 1920x1080 fp16: generate")
    w = syn.config4()
    refs = []
    for f in range(w.image.shape[0]):
        r = oracle.fill(w.image[f].astype(np.float64), w.label[f], w.guide[f], storage="f16")
        refs.append((r.shell, r.u.astype(np.float16), r.K, r.n_filled))
    banner("c4 oracle done")
    return w, refs


def _config4_launch(name, w):
    import torch

    import paper_1611_05319_amd as gf
    from paper_1611_05319_amd import autotune

    if name == "autotuned":  # the launch shape bench.py measures
        dev = torch.device("cuda:0")
        i4, l4, g4 = (torch.from_numpy(a).to(dev) for a in (w.image, w.label, w.guide))
        p = autotune.tune(i4, l4, g4, gf.Params(eps=w.eps, mu=w.mu), reps=3)
        del i4, l4, g4
        return {k: getattr(p, k) for k in ("engine", "group", "blocks_per_cu", "tile_w", "tile_h",
                                           "pass_shells", "tile_threads")}
    return dict(LAUNCH[name])


def test_config4_batched_all_frames(config4_reference):
    """Every frame of the 64-frame binary16 batch at full size, on both
    engines and on the launch shape the autotuner picks (bench.py's): the
    three give the same bits; shell maps equal the oracle's bit for bit; every
    filled value is the correctly rounded FP64 value of the fill from the
    GPU's own state at its shell (ties aside, which either rounding direction
    satisfies); against the oracle's own chained fill at most a small
    fraction of values differ, by at most 2 binary16 spacings."""
    import torch

    import paper_1611_05319_amd as gf

    w, refs = config4_reference
    dev = torch.device("cuda:0")
    i4, l4, g4 = (torch.from_numpy(a).to(dev) for a in (w.image, w.label, w.guide))
    first = None
    for launch in ("tiled", "front", "autotuned"):
        kw = _config4_launch(launch, w)
        banner(f"c4 fill launch={launch} {kw}")
        r = gf.fill_batched(i4, l4, g4, gf.Params(eps=w.eps, mu=w.mu, **kw))
        torch.cuda.synchronize()
        st = r.host_stats()
        assert not st["sync_timeout"]
        got = (r.out.cpu().numpy(), r.shell.cpu().numpy(), st)
        del r
        if first is None:
            first = got
            continue
        np.testing.assert_array_equal(got[1], first[1], err_msg=f"{launch}: shell maps")
        np.testing.assert_array_equal(got[0], first[0], err_msg=f"{launch}: colours")
        for key in ("K", "filled", "hole", "frame_K", "frame_filled", "frame_hole"):
            assert got[2][key] == first[2][key], key
    u4, s4, st = first
    differing = worst = vals = ties = 0
    for f, (rs, ru, rK, rn) in enumerate(refs):
        np.testing.assert_array_equal(s4[f], rs, err_msg=f"frame {f}")
        filled = rs >= 0
        # unfilled pixels keep their input exactly
        np.testing.assert_array_equal(u4[f][~filled], w.image[f][~filled])
        assert st["frame_K"][f] == rK and st["frame_filled"][f] == rn, f"frame {f}"
        n, t, bad = f16_one_step(w.image[f], w.label[f], w.guide[f], u4[f], s4[f], w.eps, w.mu)
        assert bad == 0, f"frame {f}: {bad} values are not the correctly rounded fill of their inputs"
        vals += n
        ties += t
        ulps = f16_ulps(u4[f][filled].astype(np.float64), ru[filled].astype(np.float64))
        differing += int((ulps > 0).sum())
        worst = max(worst, float(ulps.max()) if ulps.size else 0.0)
    total = sum(rn for _, _, _, rn in refs)
    banner(f"c4: {vals} values correctly rounded from their inputs ({ties} ties rounded the other "
           f"way); against the chained oracle fill {differing} of {3 * total} differ, at most "
           f"{worst} binary16 spacings")
    assert worst <= 2.0
    assert differing <= 1e-3 * 3 * total
    assert st["K"] == max(rK for _, _, rK, _ in refs) and st["filled"] == total


@pytest.mark.parametrize("engine", ENGINES)
def test_smart_order_threshold_on_a_straight_edge(engine):
    # the ready test of eqn:ready taken just below and just above the closed-form
    # confidence of a first-row pixel (oracle pin of the same name)
    from test_oracle_pins import _half_plane_confidence

    banner(f"smart-order threshold engine={engine}")
    H, W, eps, mu = 10, 23, 3.0, 1.0
    C0 = _half_plane_confidence(eps, mu, lambda n, m: n >= 1)
    img = np.random.default_rng(5).uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    lab = np.zeros((H, W), dtype=np.uint8)
    lab[4:] = 1
    g = np.zeros((H, W, 2), dtype=np.float32)
    g[..., 0] = 1.0
    for c in (C0 * (1 - 1e-9), C0 * (1 + 1e-9)):
        ref, u, s, st, _ = _check(img, lab, g, eps=eps, mu=mu, c=c, **LAUNCH[engine])
        assert (s[4, W // 2] == 0) == (c < C0)


@pytest.mark.parametrize("kw", [{"group": 16}, {"group": 16, "engine": 1}, {"group": 64},
                                {"group": 16, "tracking": False}])
def test_wide_ball_group_widths(kw):
    # eps = 5 (80 offsets): 16 lanes x 5 offsets, 32 x 3, 64 x 2 per lane
    banner(f"eps=5 group widths {kw}")
    rng = np.random.default_rng(21)
    img, lab, g = syn.random_tiny(rng, 90, 110, C=3, p_hole=0.4, p_bystander=0.05)
    _check(img, lab, g, eps=5.0, mu=100.0, **kw)


@pytest.mark.parametrize("engine", ENGINES)
def test_more_frames_than_lds_statistics(engine):
    # 70 small frames: the frames past the 64 with LDS statistics accumulators
    # count through global atomics; every frame's map and statistics must
    # equal its own single-frame fill
    banner(f"70 frames engine={engine}")
    rng = np.random.default_rng(70)
    frames = [syn.random_tiny(rng, 24, 30, C=3, p_hole=rng.uniform(0.0, 0.7), p_bystander=0.05)
              for _ in range(70)]
    bi = np.stack([f[0] for f in frames])
    bl = np.stack([f[1] for f in frames])
    bg = np.stack([f[2] for f in frames])
    ub, sb, stb, _ = gpu_fill(bi, bl, bg, **LAUNCH[engine])
    K = 0
    for i, (fi, fl, fg) in enumerate(frames):
        ref = oracle.fill(fi, fl, fg)
        np.testing.assert_array_equal(sb[i], ref.shell)
        assert_colour_parity(ub[i], ref.u, ref.shell)
        assert stb["frame_K"][i] == ref.K
        assert stb["frame_filled"][i] == ref.n_filled
        assert stb["frame_hole"][i] == int((fl == 1).sum())
        K = max(K, ref.K)
    assert stb["K"] == K
