"""Golden-section line search (the lambda search of Sec. 3.2) on known
unimodal functions; no GPU needed."""
import math

import pytest

from paper_2108_01438_amd.tune import INV_PHI, golden_section_max


@pytest.mark.parametrize("peak", [-3.2, -2.0, -0.9, -0.51])
def test_finds_the_maximum_of_a_unimodal_function(peak):
    f = lambda u: 1.0 - (u - peak) ** 2          # noqa: E731
    u, v, hist = golden_section_max(f, -3.5, -0.5, 20)
    assert len(hist) == 22
    assert abs(u - peak) <= 3.0 * INV_PHI ** 20 + 1e-12
    assert v == max(h[1] for h in hist)


def test_interval_shrinks_by_the_golden_ratio():
    seen = []
    golden_section_max(lambda u: (seen.append(u), -abs(u - 0.3))[1], 0.0, 1.0, 6)
    # the first two probes split [0, 1] in golden proportion, and each later
    # probe reuses one of the previous pair
    assert seen[0] == pytest.approx(1.0 - INV_PHI)
    assert seen[1] == pytest.approx(INV_PHI)
    assert len(set(round(s, 12) for s in seen)) == len(seen)


def test_flat_and_edge_maxima():
    u, v, _ = golden_section_max(lambda u: 5.0, 0.0, 1.0, 5)
    assert v == 5.0 and 0.0 <= u <= 1.0
    u, v, _ = golden_section_max(lambda u: u, 0.0, 1.0, 30)     # maximum at the right edge
    assert u == pytest.approx(1.0, abs=1e-5)
    u, v, _ = golden_section_max(lambda u: -math.exp(u), -2.0, 2.0, 30)   # left edge
    assert u == pytest.approx(-2.0, abs=1e-5)
