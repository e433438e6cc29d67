"""Host logic of the learned-theta calibration (no GPU): the bisection and
the interpolation of interactions to exactly the target error."""
import math

import pytest

from paper_0909_0541_amd import learned


def test_bisect_meets_a_tight_band():
    # a monotone error curve like the RMS error's growth with theta
    f = lambda th: 1e-3 * (th / 0.42) ** 3.5
    x, y = learned.bisect(f, 0.3, 1.0, 1e-3)
    assert abs(y / 1e-3 - 1) <= 0.003
    assert x == pytest.approx(0.42, rel=1e-3)


def test_bisect_returns_the_end_when_the_target_is_out_of_reach():
    f = lambda th: 1e-3 * (th / 0.42) ** 3.5
    assert learned.bisect(f, 0.3, 1.0, 1e-9)[0] == 0.3
    assert learned.bisect(f, 0.3, 1.0, 1.0)[0] == 1.0


def test_at_target_interpolates_between_the_bracketing_evaluations():
    # interactions ~ theta^-3, error ~ theta^3.5: a power law in the error
    hist = [(th, 1e-3 * (th / 0.42) ** 3.5, int(1e10 * (0.42 / th) ** 3)) for th in (0.3, 0.4, 0.45, 0.6)]
    got = learned.at_target(hist, 1e-3)
    assert got == pytest.approx(1e10, rel=1e-6)  # exact for a power law in log-log
    assert learned.at_target([h for h in hist if h[1] < 1e-3], 1e-3) is None
    assert learned.at_target([h for h in hist if h[1] > 1e-3], 1e-3) is None


def test_at_target_uses_the_closest_pair():
    hist = [(0.3, 5e-4, 300), (0.41, 9.9e-4, 101), (0.43, 1.01e-3, 99), (0.6, 3e-3, 50)]
    got = learned.at_target(hist, 1e-3)
    assert 99 < got < 101
    t = (math.log(1e-3) - math.log(9.9e-4)) / (math.log(1.01e-3) - math.log(9.9e-4))
    assert got == pytest.approx(math.exp(math.log(101) + t * (math.log(99) - math.log(101))))
