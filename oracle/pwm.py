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

Start-up ramp (Sec. 3.3, nonlinear model): the source is multiplied by
alpha(t) = (1 - cos(pi t / (R T))) / 2 for t < R T and by 1 afterwards, with
T = 1/f and R = 2 periods.  The printed argument lacks the period; read
literally (t in seconds) the factor would stay below 0.002 for the whole
simulated time, so it is read as rising from 0 to 1 over the first R periods.

Ties.  With the reference amplitude equal to the carrier peak, the time
grids of the workloads hit r(t) = c(t) exactly (t = T/4: r_A = 1 = c), where
the sign of a difference of two rounded values is decided by the last ulp of
the sine.  A difference within TIE_BAND = 1e-12 of zero is therefore read as
a tie (sgn = 0).  Every other decision on the workload grids has a margin
above 1e-7, so the band changes nothing else.
"""

import math
import numpy as np

TIE_BAND = 1e-12


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
    d = reference(t, src, phase_index) - carrier(t, src.f_carrier, src.carrier)
    return np.where(np.abs(d) <= TIE_BAND, 0.0, np.sign(d))


def ramp(t, src):
    """Start-up factor alpha(t) of the nonlinear model (1 when src.ramp_periods = 0),
    at the shifted time t_start + t."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64)) + getattr(src, "t_start", 0.0)
    if src.ramp_periods <= 0:
        return np.ones_like(t)
    span = src.ramp_periods / src.freq
    return np.where(t < span, 0.5 * (1.0 - np.cos(math.pi * t / span)), 1.0)


def phase_signals(t, src):
    """[3, len(t)] array of b_p(t); with src.signal == "sine" the sine
    references r_p(t) themselves (the smooth source that drives the
    nested-iteration start, Sec. 4.1).  Sampled at the shifted time t_start + t."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64)) + getattr(src, "t_start", 0.0)
    if getattr(src, "signal", "pwm") == "sine":
        return np.stack([reference(t, src, p) for p in range(3)])
    return np.stack([pwm(t, src, p) for p in range(3)])
