"""The product's target-SNR rule (paper_2110_13115_amd/tuning.py, host code)
against the oracle's (Eq. target_snr_criteria).  CPU only."""
import numpy as np

from oracle import hier as oh
from paper_2110_13115_amd import tuning


def test_target_snr_matches_oracle():
    rng = np.random.default_rng(5)
    grid = np.arange(4.0, 8.0, 0.05)
    for _ in range(200):
        flat = 4.0 + rng.exponential(1.0, size=rng.integers(0, 300))
        keep = rng.random(flat.shape[0]) < rng.uniform(0.5, 1.0)
        # lost triggers are the low ones more often, as averaging loses weak peaks
        keep |= flat > rng.uniform(4.5, 7.0)
        fin = flat[keep] * (1 + 1e-3 * rng.standard_normal(int(keep.sum())))
        for ratio in (0.9, 0.99, 0.995):
            assert tuning.target_snr(fin, flat, grid, ratio) == oh.target_snr(fin, flat, grid, ratio)


def test_target_snr_edges():
    assert tuning.target_snr([], [], [5.0, 6.0]) == 5.0            # nothing to keep: holds at once
    assert tuning.target_snr([], [5.5], [5.0, 6.0]) == 6.0
    assert tuning.target_snr([], [6.5], [5.0, 6.0]) == float("inf")
