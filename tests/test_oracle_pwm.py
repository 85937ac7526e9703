"""Pins of the oracle's PWM excitation (Sec. 3.2, Sec. 3.3 reference/carrier equations)."""

import math

import numpy as np
import pytest

from workload import Source
from oracle import pwm

FC = 20.0e3


@pytest.mark.parametrize("kind", ["triangle", "sawtooth"])
@pytest.mark.parametrize("level", [-0.9, -0.35, 0.0, 0.5, 0.8])
def test_duty_cycle_mean_equals_reference(kind, level):
    """Over one carrier period, the mean of sgn(r - c) equals r for a constant
    reference |r| <= 1 (the defining property of PWM: the time average follows
    the reference)."""
    n = 400000
    t = (np.arange(n) + 0.5) / n / FC
    b = np.sign(level - pwm.carrier(t, FC, kind))
    assert b.mean() == pytest.approx(level, abs=5e-5)


def test_carrier_hand_values():
    T = 1.0 / FC
    tri = lambda t: float(pwm.carrier(t, FC, "triangle"))
    saw = lambda t: float(pwm.carrier(t, FC, "sawtooth"))
    assert tri(0.0) == 1.0
    assert tri(T / 4) == pytest.approx(0.0, abs=1e-12)
    assert tri(T / 2) == pytest.approx(-1.0, abs=1e-12)
    assert tri(3 * T / 4) == pytest.approx(0.0, abs=1e-12)
    assert tri(T / 8) == pytest.approx(0.5, abs=1e-12)
    assert saw(0.0) == -1.0
    assert saw(T / 2) == pytest.approx(0.0, abs=1e-12)
    assert saw(T / 4) == pytest.approx(-0.5, abs=1e-12)
    assert saw(0.999 * T) == pytest.approx(0.998, abs=1e-9)


def test_three_phase_values():
    src = Source()
    # t = 0: r = (0, sin(-2pi/3), sin(-4pi/3)) = (0, -0.866, +0.866), c = 1 -> all -1
    assert pwm.phase_signals([0.0], src)[:, 0].tolist() == [-1.0, -1.0, -1.0]
    # t = T_c/4: c = 0, r_A = sin(2 pi 50 * 12.5us) > 0
    t = 0.25 / FC
    assert pwm.phase_signals([t], src)[:, 0].tolist() == [1.0, -1.0, 1.0]
    # balanced references sum to zero
    tt = np.linspace(0, 0.02, 101)
    rs = sum(pwm.reference(tt, src, p) for p in range(3))
    assert np.abs(rs).max() < 1e-12


def test_sign_of_zero_is_zero():
    # reference crossing the carrier exactly: sgn(0) = 0
    src = Source(phases=(math.pi / 2, 0.0, 0.0), carrier="triangle")
    # r_A(0) = sin(pi/2) = 1 = c(0)
    assert pwm.pwm(0.0, src, 0) == 0.0


def test_quarter_period_tie_is_zero():
    """At t = T/4 the phase-A reference peaks at 1 where the triangle carrier
    also peaks at 1: an exact tie, sgn = 0 regardless of the sine's last ulp."""
    src = Source()
    t = 0.25 / src.freq
    assert pwm.pwm(t, src, 0) == 0.0
    assert pwm.pwm(np.nextafter(t, 1.0), src, 0) == 0.0


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg4"])
def test_tie_band_changes_no_other_decision(name):
    """Outside the exact ties, |r - c| on every level's time grid is far above
    the tie band, so the band only resolves genuine ties."""
    from workload import config
    cfg = config(name)
    for l in range(cfg.n_levels):
        t = np.arange(cfg.level_steps(l) + 1) * cfg.level_dt(l)
        for p in range(3):
            d = np.abs(pwm.reference(t, cfg.source, p) - pwm.carrier(t, cfg.source.f_carrier, cfg.source.carrier))
            assert np.all((d <= 1e-14) | (d > 1e-6))


def test_startup_ramp_closed_form():
    """alpha(t) = (1 - cos(pi t / (2T))) / 2 over the first two periods, then 1."""
    src = Source(ramp_periods=2.0)
    T = 1.0 / src.freq
    t = np.array([0.0, T / 2, T, 1.5 * T, 2 * T, 3 * T])
    want = [0.0, (1 - math.cos(math.pi / 4)) / 2, 0.5, (1 - math.cos(3 * math.pi / 4)) / 2, 1.0, 1.0]
    assert np.allclose(pwm.ramp(t, src), want, rtol=0, atol=1e-15)
    assert np.all(pwm.ramp(t, Source()) == 1.0)


def test_ramp_scales_each_column_of_the_forcing():
    from workload import polar_mesh
    from oracle.stepping import Level
    mesh = polar_mesh(4, 16)
    t = np.array([1e-3, 7e-3, 0.019, 0.031, 0.05])
    f_ramp = Level(mesh, 1e-4, Source(ramp_periods=2.0)).forcing(t)
    f_flat = Level(mesh, 1e-4, Source()).forcing(t)
    want = pwm.ramp(t, Source(ramp_periods=2.0))[:, None] * f_flat
    assert np.allclose(f_ramp, want, rtol=1e-14, atol=0)
    assert np.all(f_ramp[-1] == f_flat[-1])
