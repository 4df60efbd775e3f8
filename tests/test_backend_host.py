"""Host-side EER of the library (ivx_eer) against the oracle's definition,
ties included (no GPU needed)."""
import numpy as np

from oracle import backend as be
from paper_1906_08556_amd import ivx


def test_eer_matches_the_oracle_definition():
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(2, 300))
        s = np.round(rng.standard_normal(n) * 2, int(rng.integers(0, 3))).astype(np.float32)
        t = rng.random(n) < rng.uniform(0.1, 0.9)
        if t.all() or not t.any():
            continue
        assert abs(ivx.eer(s, t) - be.eer(s.astype(np.float64), t)) < 1e-12


def test_eer_special_cases():
    assert ivx.eer(np.array([3, 4, 5, 0, 1, 2], np.float32), np.array([1, 1, 1, 0, 0, 0])) == 0.0
    assert ivx.eer(np.array([0, 1, 2, 3, 4, 5], np.float32), np.array([1, 1, 1, 0, 0, 0])) == 1.0
    assert ivx.eer(np.ones(6, np.float32), np.array([1, 0, 1, 0, 1, 0])) == 0.5
