"""Pins of the oracle's reverse-mode derivative.

The fill is linear in the known colours (Algorithm 1: every filled value is a
weighted average of values that are themselves averages of known colours), so
(i) impulse responses give the matrix A with u_out = A u_in, whose filled rows
are non-negative and sum to one, and whose transpose the adjoint must
reproduce; (ii) central finite differences in FP64 on the forward fill give the
derivative with respect to known colours exactly up to rounding, and with
respect to the guide wherever the readable sets do not change inside the
difference interval."""

import math

import numpy as np
import pytest

import oracle
import synthetic as syn


def _tiny(seed, H=9, W=10, C=1):
    rng = np.random.default_rng(seed)
    img, lab, g = syn.random_tiny(rng, H, W, C=C, p_hole=0.4, p_bystander=0.1)
    return img.astype(np.float64), lab, g.astype(np.float64)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("ghost", [True, False])
def test_impulse_matrix_and_adjoint_transpose(seed, ghost):
    img, lab, g = _tiny(seed)
    H, W, _ = img.shape
    base = oracle.fill(img, lab, g, eps=3.0, mu=10.0, ghost=ghost)
    filled = base.shell >= 0
    assert filled.any()
    known = np.argwhere(lab != 1)
    A = np.zeros((H * W, H * W))
    for (y, x) in np.argwhere(np.ones((H, W), bool)):
        e = np.zeros_like(img)
        e[y, x, 0] = 1.0
        r = oracle.fill(e, lab, g, eps=3.0, mu=10.0, ghost=ghost)
        np.testing.assert_array_equal(r.shell, base.shell)
        A[:, y * W + x] = r.u[..., 0].ravel()
    rows = np.argwhere(filled.ravel()).ravel()
    assert (A[rows] >= 0).all()
    np.testing.assert_allclose(A[rows].sum(axis=1), 1.0, atol=1e-12)
    # filled values do not depend on hole or bystander input colours
    cols_unused = np.array([y * W + x for (y, x) in np.argwhere(lab != 0)])
    assert np.abs(A[np.ix_(rows, cols_unused)]).max() == 0.0
    # A u_in reproduces the forward
    np.testing.assert_allclose(A @ img[..., 0].ravel(), base.u[..., 0].ravel(), atol=1e-12)
    # the adjoint is A^T
    rng = np.random.default_rng(seed)
    omega = rng.normal(size=(H, W, 1))
    gi, _ = oracle.adjoint(lab, g, base.u, base.shell, omega, eps=3.0, mu=10.0, ghost=ghost)
    np.testing.assert_allclose(gi[..., 0].ravel(), A.T @ omega[..., 0].ravel(), atol=1e-12)
    assert len(known) > 0


def _band_problem(seed, H=48, W=48):
    """Reduced-size differentiable workload: wiggly bands, smooth angle field."""
    rng = np.random.default_rng([seed, 0])
    img = syn.smooth_image(rng, H, W, 3, n_edges=4).astype(np.float64)
    lab = syn.wiggly_bands(rng, H, W, 2, 6.0, 10.0)
    theta = syn.smooth_angle_field(rng, H, W).astype(np.float64)
    return img, lab, theta


def _guide(theta, lab):
    g = np.stack([np.cos(theta), np.sin(theta)], -1)
    return np.where((lab == 1)[..., None], g, 0.0)


@pytest.mark.parametrize("seed", [0, 1])
def test_known_pixel_gradients_by_central_differences(seed):
    img, lab, theta = _band_problem(seed)
    g = _guide(theta, lab)
    rng = np.random.default_rng(seed + 10)
    omega = rng.normal(size=img.shape)
    fwd = oracle.fill(img, lab, g, eps=3.0, mu=50.0)
    gi, _ = oracle.adjoint(lab, g, fwd.u, fwd.shell, omega, eps=3.0, mu=50.0)
    # probes: known pixels within r + 1 of the hole, and far ones
    from scipy import ndimage
    near = ndimage.binary_dilation(lab == 1, iterations=4) & (lab == 0)
    cand = np.argwhere(near)
    picks = cand[rng.choice(len(cand), size=16, replace=False)]
    h = 1e-6
    for (y, x) in picks:
        ch = int(rng.integers(0, 3))
        p, m = img.copy(), img.copy()
        p[y, x, ch] += h
        m[y, x, ch] -= h
        Lp = float((omega * oracle.fill(p, lab, g, eps=3.0, mu=50.0).u).sum())
        Lm = float((omega * oracle.fill(m, lab, g, eps=3.0, mu=50.0).u).sum())
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gi[y, x, ch]) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("ghost", [True, False])
def test_guide_angle_gradients_by_central_differences(seed, ghost):
    img, lab, theta = _band_problem(seed)
    g = _guide(theta, lab)
    rng = np.random.default_rng(seed + 20)
    omega = rng.normal(size=img.shape)
    mu = 50.0 if ghost else 5.0
    fwd = oracle.fill(img, lab, g, eps=3.0, mu=mu, ghost=ghost)
    _, gg = oracle.adjoint(lab, g, fwd.u, fwd.shell, omega, eps=3.0, mu=mu, ghost=ghost)
    cand = np.argwhere(fwd.shell >= 0)
    rng.shuffle(cand)
    h = 1e-6
    checked = 0
    for (y, x) in cand:
        if checked == 16:
            break
        vals = []
        for d in (-h, 0.0, h):
            t2 = theta.copy()
            t2[y, x] += d
            r = oracle.fill(img, lab, _guide(t2, lab), eps=3.0, mu=mu, ghost=ghost)
            if not np.array_equal(r.shell, fwd.shell):
                break
            vals.append(float((omega * r.u).sum()))
        if len(vals) != 3:
            continue
        left, right = (vals[1] - vals[0]) / h, (vals[2] - vals[1]) / h
        if abs(left - right) > 1e-3 * max(1.0, abs(left)):
            continue  # a ghost point crossed a lattice line inside the interval
        fd = (vals[2] - vals[0]) / (2 * h)
        th = theta[y, x]
        an = gg[y, x, 0] * (-math.sin(th)) + gg[y, x, 1] * math.cos(th)
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(fd)), (y, x, fd, an)
        checked += 1
    assert checked >= 12


def test_guide_magnitude_gradient_by_central_differences():
    # d/d|g| acts through the weights only (eqn:weight uses the unnormalised g)
    img, lab, theta = _band_problem(3)
    rng = np.random.default_rng(33)
    mag = rng.uniform(0.05, 0.3, size=lab.shape)
    g = _guide(theta, lab) * mag[..., None]
    omega = rng.normal(size=img.shape)
    fwd = oracle.fill(img, lab, g, eps=3.0, mu=50.0)
    _, gg = oracle.adjoint(lab, g, fwd.u, fwd.shell, omega, eps=3.0, mu=50.0)
    cand = np.argwhere(fwd.shell >= 0)
    rng.shuffle(cand)
    h = 1e-7
    for (y, x) in cand[:10]:
        for comp in (0, 1):
            vals = []
            for d in (-h, h):
                g2 = g.copy()
                g2[y, x, comp] += d
                vals.append(float((omega * oracle.fill(img, lab, g2, eps=3.0, mu=50.0).u).sum()))
            fd = (vals[1] - vals[0]) / (2 * h)
            assert abs(fd - gg[y, x, comp]) <= 2e-6 * max(1.0, abs(fd)), (y, x, comp, fd, gg[y, x, comp])
