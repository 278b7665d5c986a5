"""Pins of the oracle's PSNR (peak 2 = the [-1, 1] range, unclamped, MSE over
every value) by hand-computed values: every "PSNR vs oracle" figure and the
PSNR floors of the reduced-precision tests depend on it."""
import math

import numpy as np

from oracle import tokenizer as O


def test_constant_error_gives_forty_db():
    # MSE = 0.02^2 = 4e-4, peak^2 = 4: 10 log10(4 / 4e-4) = 10 log10(1e4) = 40 dB
    a = np.zeros((2, 3, 4, 5, 3))
    assert abs(O.psnr(a + 0.02, a) - 40.0) < 1e-9
    assert abs(O.psnr(a, a - 0.02) - 40.0) < 1e-9


def test_mixed_errors_hand_computed():
    # errors (0.2, -0.2, 0, 0): MSE = 0.08 / 4 = 0.02, 10 log10(4 / 0.02) = 10 log10(200)
    a = np.array([0.5, -0.3, 0.1, 0.9])
    b = np.array([0.3, -0.1, 0.1, 0.9])
    assert abs(O.psnr(a, b) - 23.010299956639813) < 1e-9
    # MSE over every value: the same errors in a (2, 2) array give the same figure
    assert abs(O.psnr(a.reshape(2, 2), b.reshape(2, 2)) - 23.010299956639813) < 1e-9


def test_peak_and_symmetry():
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(1000), rng.standard_normal(1000)
    p2 = O.psnr(a, b)
    assert p2 == O.psnr(b, a)
    # halving the peak costs 20 log10(2) dB
    assert abs((p2 - O.psnr(a, b, peak=1.0)) - 20.0 * math.log10(2.0)) < 1e-9
    # doubling every error costs the same 20 log10(2) dB
    assert abs((p2 - O.psnr(a, a + 2.0 * (b - a))) - 20.0 * math.log10(2.0)) < 1e-9


def test_identical_is_infinite_and_no_clamping():
    a = np.linspace(-3.0, 3.0, 11)  # values outside [-1, 1] are compared as they are
    assert O.psnr(a, a) == float("inf")
    b = a.copy()
    b[0] = -5.0  # one error of 2 over 11 values: MSE = 4 / 11
    assert abs(O.psnr(a, b) - 10.0 * math.log10(11.0)) < 1e-9
