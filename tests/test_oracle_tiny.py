"""The C oracle against the independent set-based Python transcription of
Algorithm 1 on tiny random domains (holes touching the border, bystanders,
zero and non-unit guide vectors, both neighbourhoods, onion and smart order).
Shell maps must agree exactly and colours to 1e-12."""

import numpy as np
import pytest

import oracle
import synthetic as syn
from oracle import tiny


@pytest.mark.parametrize("seed", list(range(24)))
def test_c_oracle_matches_set_transcription(seed):
    rng = np.random.default_rng(1000 + seed)
    H, W = (int(v) for v in rng.integers(6, 20, size=2))
    img, lab, g = syn.random_tiny(rng, H, W, C=2, p_hole=float(rng.uniform(0.2, 0.6)),
                                  p_bystander=float(rng.uniform(0.0, 0.2)),
                                  blob=bool(seed % 2))
    ghost = seed % 3 != 0
    c = -1.0 if seed % 4 < 2 else float(rng.choice([0.0, 0.05, 0.3]))
    mu = float(rng.choice([2.0, 10.0, 50.0, 100.0]))
    eps = float(rng.choice([2.0, 3.0, 3.6, 5.0]))
    r = oracle.fill(img, lab, g, eps=eps, mu=mu, c=c, ghost=ghost)
    tu, ts, tK = tiny.fill(img, lab, g, eps=eps, mu=mu, c=c, ghost=ghost)
    np.testing.assert_array_equal(np.array(ts, dtype=np.int32), r.shell)
    assert tK == r.K
    np.testing.assert_allclose(np.array(tu), r.u, rtol=0, atol=1e-12)


def test_lattice_line_angles_match_transcription():
    # guide angles whose ghost points fall on lattice lines (0, 30, 45, 90 deg)
    rng = np.random.default_rng(5)
    H, W = 16, 18
    img, lab, g = syn.random_tiny(rng, H, W, C=1, p_hole=0.5, p_bystander=0.05)
    angles = np.deg2rad(np.array([0.0, 30.0, 45.0, 90.0, 150.0, 270.0]))
    pick = rng.integers(0, len(angles), size=(H, W))
    g = np.stack([np.cos(angles[pick]), np.sin(angles[pick])], -1).astype(np.float32)
    g = np.where((lab == 1)[..., None], g, np.float32(0))
    for c in (-1.0, 0.05):
        r = oracle.fill(img, lab, g, eps=3.0, mu=50.0, c=c)
        tu, ts, tK = tiny.fill(img, lab, g, eps=3.0, mu=50.0, c=c)
        np.testing.assert_array_equal(np.array(ts, dtype=np.int32), r.shell)
        np.testing.assert_allclose(np.array(tu), r.u, rtol=0, atol=1e-12)
