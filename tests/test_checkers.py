"""Pins of the comparison helpers every parity test relies on (CPU only).

oracle.log_k_errors turns two arrays of ln K into elementwise errors and
gpu_helpers.log_close applies the log-domain bars (max and median) to them.
If either silently returned 0 or True for a bad input, every 784-qubit
parity test would pass vacuously, so each planted mistake below (a one-sided
-inf, a NaN, an error that only the median or only the maximum catches) must
be rejected, and values that meet the bars must be accepted."""

import math

import numpy as np
import pytest

from oracle import checks
from gpu_helpers import LOG_TOL_MAX, LOG_TOL_MEDIAN, log_close


def test_log_k_errors_plain_differences():
    a = np.array([-1.0, -200.5, 0.0, -3.25])
    b = np.array([-1.5, -200.0, -1e-3, -3.25])
    assert np.array_equal(checks.log_k_errors(a, b), [0.5, 0.5, 1e-3, 0.0])
    # symmetric in its arguments
    assert np.array_equal(checks.log_k_errors(b, a), checks.log_k_errors(a, b))


def test_log_k_errors_exact_zeros_on_both_sides_agree():
    a = np.array([-np.inf, -np.inf])
    assert np.array_equal(checks.log_k_errors(a, a), [0.0, 0.0])


@pytest.mark.parametrize("a,b", [(-np.inf, -5.0), (-5.0, -np.inf), (np.inf, -5.0), (-np.inf, np.inf)])
def test_log_k_errors_one_sided_infinity_is_an_infinite_error(a, b):
    # an exact zero on one side only (or a blow-up) must never count as a match
    e = checks.log_k_errors(np.array([a, -1.0]), np.array([b, -1.0]))
    assert math.isinf(e[0]) and e[0] > 0
    assert e[1] == 0.0
    assert not log_close(e)


def test_log_k_errors_propagates_nan():
    e = checks.log_k_errors(np.array([np.nan, -1.0]), np.array([-1.0, -1.0]))
    assert math.isnan(e[0])
    assert not log_close(e)
    e = checks.log_k_errors(np.array([-1.0]), np.array([np.nan]))
    assert not log_close(e)


def test_log_close_accepts_errors_within_both_bars():
    rng = np.random.default_rng(0)
    e = np.concatenate([rng.uniform(0, LOG_TOL_MEDIAN, 999), [LOG_TOL_MAX]])
    assert log_close(e)
    assert log_close(np.zeros(0))  # nothing to compare


def test_log_close_rejects_a_median_over_its_bar_when_the_max_passes():
    # every error 2e-4: the max bar (5e-3) alone would pass
    e = np.full(1000, 4 * LOG_TOL_MEDIAN)
    assert e.max() <= LOG_TOL_MAX
    assert not log_close(e)


def test_log_close_rejects_one_outlier_when_the_median_passes():
    e = np.zeros(1000)
    e[17] = 2 * LOG_TOL_MAX
    assert np.median(e) <= LOG_TOL_MEDIAN
    assert not log_close(e)


def test_log_close_flattens_its_input():
    e = np.zeros((10, 10))
    e[3, 4] = 1.0
    assert not log_close(e)


def test_check_gram_pins():
    rng = np.random.default_rng(1)
    G = rng.normal(size=(6, 4)) + 1j * rng.normal(size=(6, 4))
    G /= np.linalg.norm(G, axis=1, keepdims=True)
    K = np.abs(G.conj() @ G.T) ** 2  # a valid kernel Gram
    assert checks.check_gram(K) == {}
    bad = K.copy()
    bad[0, 1] += 1e-6  # asymmetric
    assert "symmetry" in checks.check_gram(bad)
    bad = K.copy()
    bad[2, 2] = 0.99
    assert "diag" in checks.check_gram(bad)
    bad = K.copy()
    bad[1, 3] = bad[3, 1] = 1.5
    assert "range" in checks.check_gram(bad)
    # symmetric, unit diagonal, entries in [0, 1], but not PSD
    npsd = np.array([[1.0, 0.9, 0.0], [0.9, 1.0, 0.9], [0.0, 0.9, 1.0]])
    assert "psd" in checks.check_gram(npsd)
