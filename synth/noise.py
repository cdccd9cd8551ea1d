"""Poisson-Gaussian pixel-processor-array sensor noise (App. D.1).

A clean linear intensity x in [0, 1] goes through
  PRNU            x' = clip(x (1 + eta), 0, 1),        eta ~ N(0, sigma_p^2)
  electrons       n_e = Poisson(alpha F x') + Poisson(lambda_d t_e) + N(0, sigma_r^2)
  ADC             DN = clip(n_e / g, 0, 2^b - 1), rounded to an integer code,
                  output DN / (2^b - 1).
The paper writes the ADC step as a clip and calls the output quantised; the
rounding to the nearest code is this module's reading of "quantised".

theta = (alpha, sigma_r, lambda_d, sigma_p, F, g, b, t_e) with the paper's two
settings PPA_MILD and PPA_STRONG. The seeded generator is synthetic input
only: it holds none of the method's arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class SensorNoise:
    alpha: float      # exposure scale
    sigma_r: float    # read noise (electrons)
    lambda_d: float   # dark-current rate (electrons / s)
    sigma_p: float    # PRNU standard deviation
    F: float          # full-well capacity (electrons)
    g: float          # gain (electrons / DN)
    b: int            # ADC bit depth
    t_e: float        # exposure time (s)

    @property
    def full_scale(self) -> float:
        return float(2 ** self.b - 1)


PPA_STRONG = SensorNoise(0.20, 25.0, 1.0, 0.01, 15000.0, 1.5, 10, 0.001)
PPA_MILD = SensorNoise(0.12, 8.0, 0.3, 0.003, 15000.0, 1.5, 10, 0.001)


def degrade(x: np.ndarray, theta: SensorNoise, rng: np.random.Generator) -> np.ndarray:
    """One noisy exposure of the clean image x (float32 output in [0, 1])."""
    x = np.asarray(x, dtype=np.float64)
    xp = np.clip(x * (1.0 + rng.normal(0.0, theta.sigma_p, x.shape)), 0.0, 1.0)
    ne = (rng.poisson(theta.alpha * theta.F * xp).astype(np.float64) +
          rng.poisson(theta.lambda_d * theta.t_e, x.shape).astype(np.float64) +
          rng.normal(0.0, theta.sigma_r, x.shape))
    dn = np.rint(np.clip(ne / theta.g, 0.0, theta.full_scale))
    return (dn / theta.full_scale).astype(np.float32)


def expected_code(x: float, theta: SensorNoise) -> float:
    """Mean output before clipping and rounding for PRNU-free input: E[n_e] / g
    scaled to [0, 1] (used by the tests of this module)."""
    return (theta.alpha * theta.F * x + theta.lambda_d * theta.t_e) / theta.g / theta.full_scale


def code_variance(x: float, theta: SensorNoise) -> float:
    """Variance of the output for PRNU-free input away from the clip limits:
    Poisson signal + dark current + read noise, through the gain, plus the
    uniform rounding error of one code (1/12), in output units."""
    ve = theta.alpha * theta.F * x + theta.lambda_d * theta.t_e + theta.sigma_r ** 2
    return (ve / theta.g ** 2 + 1.0 / 12.0) / theta.full_scale ** 2


def render_noisy_frame(cfg, scene, cam, poses, f: int, theta: SensorNoise, keyframe: bool = False):
    """Frame f of a sequence (as render_sequence_frame, without its Gaussian
    pixel noise and occluders) through the sensor model: (image, depth,
    normals). Seeded by the sequence seed, the frame index and the setting."""
    from .scenes import render
    img, depth, nrm, _ = render(scene, cam, poses[f])
    tag = int(round(theta.alpha * 1000)) * 1000 + int(round(theta.sigma_r))
    rng = np.random.default_rng([cfg.seed, f, 1 if keyframe else 0, 7, tag])
    return degrade(img, theta, rng), depth, nrm
