"""Reverse-shell adjoint on the GPU against the oracle's adjoint (which is
itself pinned to FP64 finite differences and to the impulse matrix on the
CPU).  Per-probe error <= 1e-4 and relative L2 error <= 1e-5."""

import numpy as np
import pytest

import oracle
import synthetic as syn
from gpu_helpers import assert_colour_parity, banner, gpu_fill, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _frames(B, H, W, seed=5):
    imgs, labs, thetas = [], [], []
    for f in range(B):
        rng = np.random.default_rng([seed, f])
        imgs.append(syn.smooth_image(rng, H, W, 3, n_edges=12))
        labs.append(syn.wiggly_bands(rng, H, W, 3, 6.0, 16.0))
        thetas.append(syn.smooth_angle_field(rng, H, W))
    lab = np.stack(labs)
    th = np.stack(thetas)
    g = np.stack([np.cos(th), np.sin(th)], -1).astype(np.float32)
    g = np.where((lab == 1)[..., None], g, np.float32(0)).astype(np.float32)
    return np.stack(imgs), lab, g, th


def _compare(B, H, W, ghost=True, mu=50.0, eps=3.0, **launch):
    import torch

    import paper_1611_05319_amd as gf

    img, lab, g, th = _frames(B, H, W)
    rng = np.random.default_rng(77)
    omega = rng.normal(size=img.shape).astype(np.float32)
    u, s, st, r = gpu_fill(img, lab, g, ghost=ghost, mu=mu, eps=eps, **launch)
    gi, gg = gf.fill_backward(to_dev(omega), r, to_dev(lab), to_dev(g),
                              gf.Params(eps=eps, mu=mu, ghost=ghost))
    torch.cuda.synchronize()
    gi, gg = gi.cpu().numpy().astype(np.float64), gg.cpu().numpy().astype(np.float64)
    ref = oracle.fill(img, lab, g, eps=eps, mu=mu, ghost=ghost)
    np.testing.assert_array_equal(s, ref.shell)
    worst = assert_colour_parity(u, ref.u, ref.shell)
    banner(f"forward: K={st['K']} worst rel colour err {worst:.2e}")
    # the oracle adjoint at the oracle's own forward (nothing taken from the HIP path)
    ri, rg = oracle.adjoint(lab, g, ref.u, ref.shell, omega.astype(np.float64), eps=eps, mu=mu,
                            ghost=ghost)
    for name, a, b in (("img", gi, ri), ("guide", gg, rg)):
        err = np.abs(a - b)
        rel_l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        banner(f"grad {name}: max abs {err.max():.2e} rel L2 {rel_l2:.2e}")
        assert err.max() <= 1e-4
        assert rel_l2 <= 1e-5
    return st


@pytest.mark.parametrize("ghost", [True, False])
@pytest.mark.parametrize("eps", [3.0, 3.6, 5.0, 6.0, 9.0])  # windows of radius 3 to 9; 8 to 64 lanes
def test_adjoint_small(ghost, eps):
    banner(f"adjoint 2 x 96 x 128 ghost={ghost} eps={eps}")
    _compare(2, 96, 128, ghost=ghost, mu=50.0 if ghost else 5.0, eps=eps)


# the forward launches: each engine at its defaults, and the global front at
# 8 lanes per pixel and 2 workgroups per CU, the shape the autotuner picks for
# this workload
@pytest.mark.parametrize("launch", [{"engine": 0}, {"engine": 1},
                                    {"engine": 1, "group": 8, "blocks_per_cu": 2}],
                         ids=["tiled", "front", "front8x2"])
def test_adjoint_config5_full(launch):
    banner(f"adjoint 16 x 512 x 512, forward launch {launch}")
    st = _compare(16, 512, 512, **launch)
    assert st["K"] >= 3


@pytest.mark.parametrize("C,eps", [(1, 3.0), (2, 4.5), (4, 3.0)])
def test_adjoint_channels_bystanders_random_guides(C, eps):
    """Channel counts other than 3, ragged sizes, bystanders, zero guides
    (the lattice ball) and guides of random magnitude."""
    import torch

    import paper_1611_05319_amd as gf

    banner(f"adjoint random tiny C={C} eps={eps}")
    rng = np.random.default_rng([31, C])
    img, lab, g = syn.random_tiny(rng, 67, 101, C=C, p_hole=0.35, p_bystander=0.1)
    g = g.astype(np.float32)
    u, s, st, r = gpu_fill(img, lab, g, eps=eps)
    ref = oracle.fill(img, lab, g, eps=eps)
    np.testing.assert_array_equal(s, ref.shell)
    assert_colour_parity(u, ref.u, ref.shell)
    omega = np.random.default_rng([32, C]).normal(size=img.shape).astype(np.float32)
    gi, gg = gf.fill_backward(to_dev(omega), r, to_dev(lab), to_dev(g), gf.Params(eps=eps))
    torch.cuda.synchronize()
    gi, gg = gi.cpu().numpy().astype(np.float64), gg.cpu().numpy().astype(np.float64)
    ri, rg = oracle.adjoint(lab, g, ref.u, ref.shell, omega.astype(np.float64), eps=eps)
    for name, a, b in (("img", gi, ri), ("guide", gg, rg)):
        err = np.abs(a - b)
        rel_l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        banner(f"grad {name}: max abs {err.max():.2e} rel L2 {rel_l2:.2e}")
        assert err.max() <= 1e-4
        assert rel_l2 <= 1e-5


@pytest.mark.parametrize("order", [{"c": 0.05}, {"c2": 0.3}], ids=["smart", "ready2"])
def test_adjoint_after_other_orders(order):
    """The adjoint needs only the shell map: after a smart-order fill
    (eqn:ready) or one held back by the data term (eqn:ready2) it matches the
    oracle's adjoint at the oracle's fill in that order."""
    import torch

    import paper_1611_05319_amd as gf

    banner(f"adjoint after {order}")
    rng = np.random.default_rng(33)
    img, lab, g = syn.random_tiny(rng, 67, 101, C=3, p_hole=0.35, p_bystander=0.05)
    g = g.astype(np.float32)
    u, s, st, r = gpu_fill(img, lab, g, **order)
    ref = oracle.fill(img, lab, g, **order)
    np.testing.assert_array_equal(s, ref.shell)
    assert_colour_parity(u, ref.u, ref.shell)
    omega = np.random.default_rng(34).normal(size=img.shape).astype(np.float32)
    gi, gg = gf.fill_backward(to_dev(omega), r, to_dev(lab), to_dev(g), gf.Params(**order))
    torch.cuda.synchronize()
    gi, gg = gi.cpu().numpy().astype(np.float64), gg.cpu().numpy().astype(np.float64)
    ri, rg = oracle.adjoint(lab, g, ref.u, ref.shell, omega.astype(np.float64))
    for name, a, b in (("img", gi, ri), ("guide", gg, rg)):
        err = np.abs(a - b)
        rel_l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        banner(f"grad {name}: max abs {err.max():.2e} rel L2 {rel_l2:.2e}")
        assert err.max() <= 1e-4
        assert rel_l2 <= 1e-5


@pytest.mark.parametrize("ghost", [True, False])
def test_adjoint_binary16_storage(ghost):
    """The adjoint of a binary16-storage fill (it reads the forward's binary16
    colours) against the oracle's adjoint at the oracle's own binary16 fill.
    The two fills agree bit for bit (FP64 tensor-product values, one rounding
    to binary16 each; see the binary16 parity tests), which is asserted first,
    so both adjoints see the same colours."""
    import torch

    import paper_1611_05319_amd as gf

    banner(f"adjoint, binary16 storage, ghost={ghost}")
    img, lab, g, th = _frames(2, 96, 128, seed=11)
    img16 = img.astype(np.float16)
    mu = 50.0 if ghost else 5.0
    u, s, st, r = gpu_fill(img16.astype(np.float32), lab, g, ghost=ghost, mu=mu,
                           dtype=torch.float16)
    ref = oracle.fill(img16.astype(np.float64), lab, g, mu=mu, ghost=ghost, storage="f16")
    np.testing.assert_array_equal(s, ref.shell)
    np.testing.assert_array_equal(u, ref.u)
    omega = np.random.default_rng(79).normal(size=img.shape).astype(np.float32)
    gi, gg = gf.fill_backward(to_dev(omega), r, to_dev(lab), to_dev(g),
                              gf.Params(mu=mu, ghost=ghost))
    torch.cuda.synchronize()
    gi, gg = gi.cpu().numpy().astype(np.float64), gg.cpu().numpy().astype(np.float64)
    ri, rg = oracle.adjoint(lab, g, ref.u, ref.shell, omega.astype(np.float64), mu=mu, ghost=ghost)
    for name, a, b in (("img", gi, ri), ("guide", gg, rg)):
        err = np.abs(a - b)
        rel_l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        banner(f"grad {name}: max abs {err.max():.2e} rel L2 {rel_l2:.2e}")
        assert err.max() <= 1e-4
        assert rel_l2 <= 1e-5


def test_adjoint_replays_given_shell_count():
    """K passed explicitly (the forward's statistic) equals K taken from the
    map; a smaller K is the adjoint of a fill stopped after K shells."""
    import torch

    import paper_1611_05319_amd as gf

    banner("adjoint with explicit K")
    img, lab, g, th = _frames(2, 80, 96, seed=9)
    omega = np.random.default_rng(78).normal(size=img.shape).astype(np.float32)
    u, s, st, r = gpu_fill(img, lab, g)
    K = st["K"]
    assert K >= 4
    dev_args = (to_dev(omega), r, to_dev(lab), to_dev(g), gf.Params())
    gi_a, gg_a = gf.fill_backward(*dev_args)
    gi_b, gg_b = gf.fill_backward(*dev_args, K=K)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gi_b.cpu().numpy(), gi_a.cpu().numpy(), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(gg_b.cpu().numpy(), gg_a.cpu().numpy(), rtol=1e-5, atol=1e-6)
    # replaying K - 2 shells = the adjoint of the fill stopped after K - 2 shells
    m = K - 2
    u2, s2, st2, r2 = gpu_fill(img, lab, g, max_shells=m)
    gi_c, gg_c = gf.fill_backward(to_dev(omega), r, to_dev(lab), to_dev(g), gf.Params(), K=m)
    torch.cuda.synchronize()
    ref = oracle.fill(img, lab, g, max_shells=m)
    np.testing.assert_array_equal(s2, ref.shell)
    ri, rg = oracle.adjoint(lab, g, ref.u, ref.shell, omega.astype(np.float64))
    assert np.abs(gi_c.cpu().numpy() - ri).max() <= 1e-4
    assert np.abs(gg_c.cpu().numpy() - rg).max() <= 1e-4


def test_autograd_function():
    import torch

    import paper_1611_05319_amd as gf

    banner("autograd function")
    img, lab, g, th = _frames(2, 64, 80)
    timg = to_dev(img).requires_grad_(True)
    tth = to_dev(th).requires_grad_(True)
    tlab = to_dev(lab)
    out, shell = gf.GuidefillFn.apply(timg, tth, tlab, gf.Params(eps=3.0, mu=50.0))
    rng = np.random.default_rng(3)
    omega = to_dev(rng.normal(size=img.shape).astype(np.float32))
    (out * omega).sum().backward()
    # reference: the oracle's forward and adjoint, chained to theta; g is formed
    # in float32 as the autograd function forms it
    gnp = np.stack([np.cos(th), np.sin(th)], -1).astype(np.float32)
    gnp = np.where((lab == 1)[..., None], gnp, np.float32(0))
    ref = oracle.fill(img, lab, gnp)
    np.testing.assert_array_equal(shell.cpu().numpy(), ref.shell)
    assert_colour_parity(out.detach().cpu().numpy().astype(np.float64), ref.u, ref.shell)
    ri, rg = oracle.adjoint(lab, gnp, ref.u, ref.shell, omega.cpu().numpy().astype(np.float64))
    rth = -np.sin(th) * rg[..., 0] + np.cos(th) * rg[..., 1]
    rth = np.where(lab == 1, rth, 0.0)
    assert np.abs(timg.grad.cpu().numpy() - ri).max() <= 1e-4
    gth = tth.grad.cpu().numpy()
    assert np.abs(np.where(lab == 1, gth, 0.0) - rth).max() <= 1e-4
