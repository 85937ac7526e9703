"""Pins of the oracle's FAS-MGRIT (Algorithm 1, Sec. 2.1, Sec. 2.2).

* finite termination: exact after N_t/m (F) and N_t/(2m) (FCF) iterations
  without spatial coarsening, with the exactness front advancing by one
  (F) or two (FCF) coarse intervals per iteration;
* the ideal coarse operator (coarse propagator = m fine steps) converges in
  one iteration;
* two-level F-relaxation reproduces Parareal iterate by iterate;
* with spatial coarsening, FCF still terminates by N_t/m iterations while F
  alone does not (the stall behind the failed F-relaxation runs of Table 2).
"""

import numpy as np
import pytest

from workload import config, polar_mesh
from oracle.problem import build
from oracle import mgrit, stepping


def small_cfg(**kw):
    # 8 x 64 machine, 128 steps over 5 ms, two levels, m = 8
    base = dict(meshes=config("cfg1").meshes[:1] * 2, n_steps=128, m=8, t_final=0.005)
    base.update(kw)
    cfg = config("cfg1", **base)
    from workload.configs import LevelSpec
    cfg.meshes = [LevelSpec(8, 64)] * len(cfg.meshes)
    return cfg


def _seq(H, cfg):
    return stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), cfg.n_steps)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("gamma", [0, 1])
def test_exactness_front(gamma):
    cfg = small_cfg(gamma=gamma)
    H, _ = build(cfg)
    U = _seq(H, cfg)
    m, NT = cfg.m, cfg.n_steps // cfg.m
    step = 1 if gamma == 0 else 2
    for k in [0, 1, 3]:
        u, _, _ = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=0.0, maxit=k)
        exact_upto = (step * k + step) * m - 1          # last exact time index
        err = np.linalg.norm(u - U, axis=1) / np.linalg.norm(U, axis=1).clip(1e-300)
        assert err[: exact_upto + 1].max() < 1e-12, (k, err[: exact_upto + 1].max())
        assert err[exact_upto + 1] > 1e-6
    # finite termination after N_T (F) or N_T/2 (FCF) corrections
    kmax = NT if gamma == 0 else NT // 2
    u, hist, _ = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=0.0, maxit=kmax)
    assert _rel(u, U) < 1e-12
    assert hist[-1] < 1e-12 * hist[0]


@pytest.mark.slow
def test_exact_after_nt_over_m_cfg1_sizes():
    """The machine and time grid of the small linear workload (16x128, 1024
    steps, m = 16): F-relaxation is exact after 64 iterations, FCF after 32."""
    for gamma, k in [(0, 64), (1, 32)]:
        cfg = config("cfg1", gamma=gamma)
        H, _ = build(cfg)
        U = _seq(H, cfg)
        u, hist, _ = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=0.0, maxit=k)
        assert _rel(u, U) < 1e-12
        assert hist[-1] < 1e-13 * hist[0]


def test_exact_coarse_propagator_one_iteration():
    cfg = small_cfg()
    H, _ = build(cfg)
    H.levels[1] = mgrit.ExactCoarse(H.levels[0], cfg.m)
    U = _seq(H, cfg)
    u, hist, conv = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=1e-12, maxit=5)
    assert len(hist) == 2 and conv
    assert hist[1] < 1e-13 * hist[0]
    assert _rel(u, U) < 1e-12


def test_two_level_f_relaxation_is_parareal():
    cfg = small_cfg(gamma=0)
    H, _ = build(cfg)
    n = H.levels[0].n
    NT = cfg.n_steps // cfg.m
    Fprop = mgrit.ExactCoarse(H.levels[0], cfg.m)     # m fine steps
    G = H.levels[1]
    para = mgrit.parareal(G, Fprop, np.zeros(n), NT, 4)
    seen = []

    def cb(it, u, rho):
        seen.append(u[:: cfg.m].copy())   # C-points entering iteration `it` (after correction it)

    mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=0.0, maxit=4, callback=cb)
    for k in range(5):
        assert np.linalg.norm(seen[k] - para[k]) <= 1e-12 * max(np.linalg.norm(para[k]), 1e-300)


def _sc_cfg(gamma):
    from workload.configs import LevelSpec
    cfg = small_cfg(gamma=gamma)
    cfg.meshes = [LevelSpec(8, 64), LevelSpec(4, 32)]
    return cfg


def test_spatial_coarsening_fcf_terminates():
    cfg = _sc_cfg(1)
    H, _ = build(cfg)
    U = _seq(H, cfg)
    NT = cfg.n_steps // cfg.m
    u, hist, _ = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=0.0, maxit=NT)
    assert _rel(u, U) < 1e-12
    assert hist[-1] < 1e-12 * hist[0]


def test_spatial_coarsening_f_relaxation_stalls():
    cfg = _sc_cfg(0)
    H, _ = build(cfg)
    U = _seq(H, cfg)
    NT = cfg.n_steps // cfg.m
    u, hist, _ = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=0.0, maxit=NT)
    assert _rel(u, U) > 1e-8
    assert hist[-1] > 1e-8 * hist[0]


@pytest.mark.parametrize("sc", [False, True])
def test_three_level_v_cycle_converges_to_sequential(sc):
    from workload.configs import LevelSpec
    cfg = small_cfg()
    cfg.meshes = ([LevelSpec(16, 128), LevelSpec(8, 64), LevelSpec(4, 32)] if sc
                  else [LevelSpec(16, 128)] * 3)
    cfg.n_steps, cfg.m = 256, 4
    H, _ = build(cfg)
    U = _seq(H, cfg)
    u, hist, conv = mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, tol=1e-8, maxit=45)
    assert conv
    assert len(hist) <= (8 if not sc else 45)
    assert _rel(u, U) < 1e-8
    # rho decreases monotonically
    assert all(b < a for a, b in zip(hist, hist[1:]))
