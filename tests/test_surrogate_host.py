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


@pytest.mark.parametrize("n,length,hw,want", [(1, 4096, 3, (256, 32)), (7, 4096, 3, (256, 24)),
                                              (9, 4096, 3, (512, 60)), (34, 4096, 3, (768, 32)),
                                              (129, 4096, 3, (0, 0)), (2, 512, 3, (256, 32)),
                                              (1, 4096, 8, (768, 32))])
def test_latency_shape_picks_the_first_shape_that_fits_one_round(n, length, hw, want):
    """Chunks per pass = n * ceil(length / (chunk - 2 hw S)) against 1.1 x 256
    compute units; a shape whose halos leave under 64 inner nodes is skipped;
    none fits -> the library's default (0, 0)."""
    assert SG.latency_shape(n, length, 256, hw=hw) == want
    c, S = want
    if c:
        assert c - 2 * hw * S >= 64
        assert n * -(-length // (c - 2 * hw * S)) <= 1.1 * 256
