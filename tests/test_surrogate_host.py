"""Host-side helpers of the surrogate rollout (no GPU): the Mach envelope
the admission check takes from the training pairs."""
import math

import pytest
import torch

from paper_1606_06107_amd import surrogate as SG


def _pairs(peaks):
    """Pairs [S][3][L] whose largest |u|/sqrt(T) is peaks[s] (T = 4 at that
    node, 1 elsewhere; rho = 1)."""
    S, L = len(peaks), 8
    x = torch.ones(S, 3, L, dtype=torch.float64)
    x[:, 1] = 0.0
    for s, p in enumerate(peaks):
        x[s, 1, 3] = 2.0 * p
        x[s, 2, 3] = 4.0
    return x


def test_envelope_is_the_largest_pair_peak_at_quantile_one():
    x = _pairs([0.5, 1.25, 0.75])
    t = _pairs([0.25, 0.5, 2.0])
    assert SG.mach_envelope(x, t, 1.0) == pytest.approx(2.0)


def test_envelope_quantile_ignores_an_extreme_pair():
    peaks = [0.5 + 0.001 * k for k in range(1000)] + [20.0]
    x = _pairs(peaks)
    env = SG.mach_envelope(x, x, 0.99)
    assert 1.3 < env < 1.6 and not math.isclose(env, 20.0)
    assert SG.mach_envelope(x, x, 1.0) == pytest.approx(20.0)
