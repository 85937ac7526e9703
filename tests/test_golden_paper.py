"""Values the paper prints (tests/golden/paper_parameters.json, each block
cited) against the workload's source settings and the oracle's PWM, and the
paper's own arithmetic between them."""

import json
import math
import os

import numpy as np

from workload import Source
from oracle import pwm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_pwm_parameters_match_the_paper():
    g = _golden()["pwm"]
    src = Source()
    assert src.freq == g["frequency_hz"]
    assert math.isclose(1.0 / src.freq, g["period_s"], rel_tol=1e-15)
    assert src.f_carrier == g["pulses_per_period"] * src.freq == g["pwm_frequency_hz"]


def test_sawtooth_carrier_is_the_printed_formula():
    """c_p(t) = 2 (p t/T - floor(p t/T)) - 1 at points strictly inside one
    carrier period (at the jumps the two products may round to either side)."""
    g = _golden()["pwm"]
    p, T = g["pulses_per_period"], g["period_s"]
    t = (np.array([0.1, 0.25, 0.5, 0.75, 0.9]) + 3.0) * T / p
    want = 2.0 * (p * t / T - np.floor(p * t / T)) - 1.0
    got = pwm.carrier(t, p / T, "sawtooth")
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    assert np.allclose(want, [-0.8, -0.5, 0.0, 0.5, 0.8], atol=1e-9)


def test_the_papers_time_grids_are_consistent():
    g = _golden()
    lin, nl = g["linear_runs"], g["nonlinear_runs"]
    assert lin["dt_s"] == 2.0 ** -20 and nl["dt_s"] == 2.0 ** -20
    assert lin["time_points"] == 2 ** 15 + 1
    assert (lin["time_points"] - 1) * lin["dt_s"] == lin["t_final_s"]
    assert (lin["time_points"] - 1) % lin["m_first_level"] == 0
    assert abs(nl["steps"] * nl["dt_s"] - nl["t_final_approx_s"]) < 3e-4


def test_figure_example_switches_at_the_carrier_frequency():
    """A sine reference of amplitude 0.8 < 1 against a sawtooth carrier: once
    per carrier period the carrier resets (b goes to +1) and once it climbs
    past the reference (b goes to -1), so b switches at the carrier rate."""
    g = _golden()["pwm_figure_example"]
    T = 1.0 / g["reference_hz"]
    n = 200_000
    t = (np.arange(n) + 0.5) * (T / n)              # one reference period, no sample on a jump
    r = g["reference_amplitude"] * np.sin(2.0 * math.pi * g["reference_hz"] * t)
    b = np.sign(r - pwm.carrier(t, g["carrier_hz"], "sawtooth"))
    assert np.all(b != 0)
    rises = np.count_nonzero((b[1:] > 0) & (b[:-1] < 0))
    falls = np.count_nonzero((b[1:] < 0) & (b[:-1] > 0))
    per_period = g["switching_hz"] * T
    assert abs(rises - per_period) <= 1 and abs(falls - per_period) <= 1
    assert abs(rises + falls - 2 * per_period) <= 1
