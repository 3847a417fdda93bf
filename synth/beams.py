"""Seeded synthetic beam weights: the phases that point beams at directions.

Discrete beamforming sums all inputs after a phase shift per input (Sec. IV-C,
"Discrete Beamforming").  The weights here stand in for a calibrated array:
inputs sit on a line with 0.3 m spacing, channel f of F is centred at
400 + 400 (f + 0.5) / F MHz (the 400-800 MHz band), beam b points at a seeded
direction with sin(theta_b) uniform in [-0.9, 0.9], and every input carries a
seeded calibration phase.  The weight of input n for beam b in channel f is
round(127 exp(-i phi)), phi = 2 pi nu_f x_n sin(theta_b) / c + cal_n, as int8
[F][B][N][2] (re, im), each in -127..127.
"""
from __future__ import annotations

import numpy as np

_KEY_BEAMS = 0xBEA


def gen_beam_weights(F: int, B: int, N: int, seed: int, amplitude: int = 127) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, _KEY_BEAMS])))
    sin_theta = rng.uniform(-0.9, 0.9, B)
    cal = rng.uniform(0.0, 2.0 * np.pi, N)
    x = 0.3 * np.arange(N)
    nu = 400e6 + 400e6 * (np.arange(F) + 0.5) / F
    phi = (2.0 * np.pi / 2.998e8) * nu[:, None, None] * sin_theta[None, :, None] * x[None, None, :]
    phi = phi + cal[None, None, :]
    w = np.empty((F, B, N, 2), np.int8)
    w[..., 0] = np.clip(np.rint(amplitude * np.cos(-phi)), -127, 127)
    w[..., 1] = np.clip(np.rint(amplitude * np.sin(-phi)), -127, 127)
    return w
