"""Pins for the oracle's H0^(1)(x) = J0(x) + i Y0(x) (the 2D Helmholtz kernel is
(i/4) H0^(1)(kappa r), section 2): against scipy's independent evaluation over
the whole range the workloads reach (kappa r up to ~150) and across the
oracle's own switch points, and against the small-argument closed forms."""
import math

import numpy as np
import pytest

import oracle

scipy_special = pytest.importorskip("scipy.special")


def test_matches_scipy_hankel1():
    x = np.concatenate([np.logspace(-10, np.log10(250.0), 5000), np.linspace(3.99, 4.01, 41),
                        np.linspace(24.99, 25.01, 41)])
    h = oracle.h0(x)
    ref = scipy_special.hankel1(0, x)
    err = np.abs(h - ref) / np.abs(ref)
    assert err.max() <= 1e-13, (err.max(), x[err.argmax()])


def test_small_argument_closed_forms():
    for x in (1e-9, 1e-7, 1e-5):
        h = oracle.h0(np.array([x]))[0]
        j0 = 1.0 - x * x / 4.0
        y0 = (2.0 / math.pi) * ((math.log(x / 2.0) + 0.5772156649015329) * j0 + x * x / 4.0)
        assert abs(h.real - j0) <= 1e-15
        assert abs(h.imag - y0) <= 1e-14 * abs(y0)


def test_zeros_of_j0():
    # the first zeros of J0 (and the value of Y0 there, where the Wronskian gives
    # |Y0 J1| = 2 / (pi x) and J1 = -J0'; checked through scipy's J1)
    zeros = np.array([2.404825557695773, 5.520078110286311, 8.653727912911013, 30.634606468431976])
    h = oracle.h0(zeros)
    assert np.max(np.abs(h.real)) <= 1e-14
    j1 = scipy_special.j1(zeros)
    np.testing.assert_allclose(h.imag * j1, 2.0 / (np.pi * zeros), rtol=1e-12)
