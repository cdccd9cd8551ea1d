"""The sensor-noise generator (App. D.1) against the moments the model fixes.

For PRNU-free input away from the clip limits, the electron count has mean
alpha F x + lambda_d t_e and variance alpha F x + lambda_d t_e + sigma_r^2
(sum of two Poisson and one Gaussian variable); the gain divides both by g and
g^2, and rounding to a code adds 1/12 code^2 of variance.
"""

import dataclasses

import numpy as np
import pytest

from synth import PPA_MILD, PPA_STRONG, degrade
from synth.noise import code_variance, expected_code


@pytest.mark.parametrize("theta", [PPA_MILD, PPA_STRONG])
@pytest.mark.parametrize("x", [0.1, 0.3])
def test_moments_without_prnu(theta, x):
    th = dataclasses.replace(theta, sigma_p=0.0)
    rng = np.random.default_rng(0)
    y = degrade(np.full(400_000, x), th, rng).astype(np.float64)
    m, v = expected_code(x, th), code_variance(x, th)
    se = np.sqrt(v / y.size)
    assert abs(y.mean() - m) < 5 * se
    assert abs(y.var() / v - 1.0) < 0.02


def test_prnu_scales_the_signal_variance():
    # multiplicative PRNU adds (alpha F x sigma_p)^2 electrons^2 of variance
    th = dataclasses.replace(PPA_STRONG, sigma_p=0.05)
    x = 0.2
    rng = np.random.default_rng(1)
    y = degrade(np.full(400_000, x), th, rng).astype(np.float64)
    extra = (th.alpha * th.F * x * th.sigma_p) ** 2 / th.g ** 2 / th.full_scale ** 2
    assert abs(y.var() / (code_variance(x, th) + extra) - 1.0) < 0.03


def test_saturation_and_range():
    # strong exposure saturates the ADC earlier than mild (Sec. D.1)
    rng = np.random.default_rng(2)
    x = np.full(10_000, 0.6)
    ys = degrade(x, PPA_STRONG, rng)
    ym = degrade(x, PPA_MILD, rng)
    assert ys.max() == 1.0 and np.mean(ys == 1.0) > 0.99
    assert np.mean(ym == 1.0) == 0.0
    assert ys.dtype == np.float32 and ys.min() >= 0.0
    # outputs are codes of the 10-bit ADC
    codes = ym.astype(np.float64) * 1023.0
    assert np.abs(codes - np.rint(codes)).max() < 1e-3
