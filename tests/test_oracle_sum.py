"""The oracle's compensated summation against a correctly rounded sum."""
import math

import numpy as np

import oracle as O


def test_compensated_sum_matches_fsum():
    rng = np.random.default_rng(2)
    for scale in (1.0, 1e8, 1e-8):
        v = rng.normal(size=100_000) * scale
        v = np.concatenate([v, [1e16, 1.0, -1e16]])        # cancellation that a plain sum loses
        exact = math.fsum(v)
        assert abs(O.compensated_sum(v) - exact) <= 2 * np.finfo(float).eps * abs(exact)
    assert O.compensated_sum(np.zeros(0)) == 0.0
    assert O.compensated_sum(np.array([1e100, 1.0, -1e100])) == 1.0
