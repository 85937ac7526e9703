"""PWM excitation (Sec. 3.2 and Sec. 3.3, reference-signal and carrier equations).

b(t) = sgn[r(t) - c(t)] with the sine reference r_s(t) = sin(2*pi*f*t + phi_s)
and a carrier c(t).  The phase angles are read as phi = (0, -2pi/3, -4pi/3)
(the printed third angle lost its index and the second its minus sign).

Two carriers:
  sawtooth (the paper's bipolar trailing-edge carrier):
      c(t) = 2 (f_c t - floor(f_c t)) - 1
  triangle (the carrier the workload configurations use):
      c(t) = 1 - 4 |f_c t - floor(f_c t + 1/2)|,   c(0) = 1.
sgn(0) = 0.  One carrier is shared by the three phases.
"""

import math
import numpy as np


def carrier(t, f_c, kind):
    t = np.asarray(t, dtype=np.float64)
    x = f_c * t
    if kind == "sawtooth":
        return 2.0 * (x - np.floor(x)) - 1.0
    if kind == "triangle":
        return 1.0 - 4.0 * np.abs(x - np.floor(x + 0.5))
    raise ValueError(kind)


def reference(t, src, phase_index):
    t = np.asarray(t, dtype=np.float64)
    phi = src.phases[phase_index] + src.phase_offset
    return np.sin(2.0 * math.pi * src.freq * t + phi)


def pwm(t, src, phase_index):
    """b_p(t) in {-1, 0, +1}."""
    return np.sign(reference(t, src, phase_index) - carrier(t, src.f_carrier, src.carrier))


def phase_signals(t, src):
    """[3, len(t)] array of b_p(t)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.stack([pwm(t, src, p) for p in range(3)])
