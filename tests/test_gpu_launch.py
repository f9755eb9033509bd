"""Persistent launches: the start-up join over a workspace's ring of join-word
sets (each call clears the next call's set), and a call that shares the
device with other work, where only the workgroups resident at start-up take
part.  The fill itself does not depend on how many workgroups take part, so
every run must reproduce the first bit for bit (and the oracle's shell map)."""

import numpy as np
import pytest

import oracle
import synthetic as syn
from gpu_helpers import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1611_05319_amd as gf

    gf.load()


LAUNCH = {"tiled": {}, "tiled256": {"tile_threads": 256}, "front": {"engine": 1}}


def _plan(w, **kw):
    import torch

    import paper_1611_05319_amd as gf

    dev = torch.device("cuda:0")
    img = torch.from_numpy(w.image).to(dev)
    lab = torch.from_numpy(w.label).to(dev)
    gd = torch.from_numpy(w.guide).to(dev)
    return gf.FillPlan(img, lab, gd, gf.Params(eps=w.eps, mu=w.mu, **kw))


def _run(plan, stream=None):
    import torch

    import paper_1611_05319_amd as gf

    plan.run(stream)
    torch.cuda.synchronize()
    st = gf.stats_fields(plan.stats)
    assert not st["sync_timeout"], "a grid barrier gave up waiting"
    assert st["workgroups"] >= 1
    return plan.out.cpu().numpy().copy(), plan.shell.cpu().numpy().copy(), st


@pytest.mark.parametrize("launch", list(LAUNCH))
def test_ring_of_join_words(launch):
    """Seven calls on one workspace walk the three join-word sets twice over."""
    w = syn.config1()
    ref = oracle.fill(w.image[0].astype(np.float64), w.label[0], w.guide[0], eps=w.eps, mu=w.mu)
    plan = _plan(w, **LAUNCH[launch])
    first = None
    for call in range(7):
        banner(f"join ring {launch} call {call}")
        u, s, st = _run(plan)
        np.testing.assert_array_equal(s[0], ref.shell)
        if first is None:
            first = (u, st["workgroups"])
        else:
            np.testing.assert_array_equal(u, first[0])
            assert st["workgroups"] == first[1]


def test_backward_ring_of_join_words():
    """The adjoint's launches walk their own workspace's ring the same way."""
    import torch

    import paper_1611_05319_amd as gf

    w = syn.config1()
    dev = torch.device("cuda:0")
    img = torch.from_numpy(w.image).to(dev)
    lab = torch.from_numpy(w.label).to(dev)
    gd = torch.from_numpy(w.guide).to(dev)
    fwd = gf.FillPlan(img, lab, gd, gf.Params(eps=w.eps, mu=w.mu))
    fwd.run()
    torch.cuda.synchronize()
    gout = torch.from_numpy(np.random.default_rng(3).standard_normal(w.image.shape).astype(np.float32)).to(dev)
    gimg = torch.empty_like(gout)
    ggd = torch.empty_like(gd)
    bwd = gf.BackwardPlan(fwd, gout, gimg, ggd)
    first = None
    for call in range(5):
        banner(f"adjoint join ring call {call}")
        bwd.run()
        torch.cuda.synchronize()
        got = (gimg.cpu().numpy().copy(), ggd.cpu().numpy().copy())
        if first is None:
            first = got
        else:
            # the scatter sums are atomic: equal up to their summation order
            np.testing.assert_allclose(got[0], first[0], rtol=1e-5, atol=1e-6)
            np.testing.assert_allclose(got[1], first[1], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("launch", list(LAUNCH))
def test_shares_the_device_with_other_work(launch):
    """A call enqueued while matrix products run on another stream: whichever
    workgroups are resident at start-up fill the frame; the result is the one
    of a call alone on the device."""
    import torch

    w = syn.config2()
    plan = _plan(w, **LAUNCH[launch])
    banner(f"alone {launch}")
    u0, s0, st0 = _run(plan)
    dev = torch.device("cuda:0")
    a = torch.randn(4096, 4096, device=dev)
    other, mine = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
    torch.cuda.synchronize()
    banner(f"beside matrix products {launch}")
    with torch.cuda.stream(other):
        for _ in range(6):
            b = a @ a
    u1, s1, st1 = _run(plan, mine)
    del b
    banner(f"workgroups alone {st0['workgroups']}, beside other work {st1['workgroups']}")
    np.testing.assert_array_equal(s1, s0)
    np.testing.assert_array_equal(u1, u0)
    assert st1["filled"] == st0["filled"] and st1["K"] == st0["K"]
