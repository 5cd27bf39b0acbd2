"""Pins of the asinh stretch oracle (Sec. 2.2.6 gray-scale maps)."""
import math

import numpy as np
import pytest

from oracle import stretch as st


def test_closed_forms():
    assert st.asinh_forward([0.0], 3.0, 2.0)[0] == 0.0
    v = np.array([1e6])
    assert st.asinh_forward(v, 30.0, 1.0)[0] == pytest.approx(
        math.log(2 * 1e6 / 30.0), rel=1e-9)
    assert st.asinh_forward([1e-6], 30.0, 2.0)[0] == pytest.approx(
        2e-6 / 30.0, rel=1e-9)


def test_derivatives_match_finite_differences():
    rng = np.random.default_rng(21)
    v = rng.normal(0, 200, 50)
    g = rng.normal(0, 1, 50)
    a, b = 30.0, 1.7
    dv, da, db = st.asinh_backward(v, g, a, b)
    h = 1e-4
    L = lambda vv, aa, bb: float(np.sum(g * st.asinh_forward(vv, aa, bb)))
    for i in range(0, 50, 7):
        e = np.zeros(50)
        e[i] = h
        fd = (L(v + e, a, b) - L(v - e, a, b)) / (2 * h)
        assert dv[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    assert da == pytest.approx((L(v, a + h, b) - L(v, a - h, b)) / (2 * h),
                               rel=1e-6)
    assert db == pytest.approx((L(v, a, b + h) - L(v, a, b - h)) / (2 * h),
                               rel=1e-6)
