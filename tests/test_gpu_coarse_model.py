"""GPU learned coarse propagator against the oracle's network (forward, manual
backward, Adam), and its use as the MGRIT coarse propagator, through the C ABI."""

import numpy as np
import pytest

from workload import config, polar_mesh
from oracle.fe import MachineFE
from oracle.problem import build
from oracle import gnn, mgrit, stepping

pytestmark = pytest.mark.gpu

MGRIT_GATE = 1e-7


def _solver(cfg, **kw):
    from paper_1912_03106_amd.solver import Solver
    return Solver(cfg, **kw)


@pytest.fixture(scope="module")
def coarse():
    """cfg1 hierarchy (16x128 on both levels): coarse step dT = 16 dt."""
    cfg = config("cfg1")
    fe = MachineFE(polar_mesh(16, 128))
    ptr, idx = gnn.graph(fe)
    flags = gnn.node_flags(fe)
    return cfg, fe, ptr, idx, flags


def _weights(m, seed, scales, out_scale=0.3):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in gnn.param_shapes(m):
        lim = np.sqrt(6.0 / (shape[0] + shape[1])) if len(shape) == 2 else 0.1
        p[name] = rng.uniform(-lim, lim, size=shape)
    p["w_out"] = rng.uniform(-out_scale, out_scale, size=(gnn.H,))
    p["scales"] = np.asarray(scales, dtype=np.float64)
    vec = gnn.pack(p, m).astype(np.float32)
    return vec, gnn.unpack(vec.astype(np.float64), m)


def _samples(cfg, fe, B, seed):
    rng = np.random.default_rng(seed)
    lev = stepping.Level(fe.mesh, cfg.level_dt(1), cfg.source, fe=fe)
    U = stepping.sequential(lev, np.zeros(fe.n), 24)
    u = U[rng.integers(4, 25, size=B)] * rng.uniform(0.5, 1.5, size=(B, 1))
    k = rng.integers(0, cfg.level_steps(1), size=B)
    p = lev.phi(u, k)
    amp = rng.uniform(0.8, 1.2, size=B)
    dphi = rng.uniform(-np.pi, np.pi, size=B)
    return u, p, k, amp, dphi


def _scales(cfg, fe, u):
    s_u = float(np.sqrt(np.mean(u * u)))
    s_f = float(cfg.source.J0 * np.max(np.abs(fe.F).sum(axis=0)))
    return [s_u, s_f, 0.05 * s_u, 0.0]


def test_forward_matches_oracle(coarse):
    """The propagator as MGRIT evaluates it (FP64 activations, bf16 weights)
    against the oracle's FP64 network with the same rounded weights."""
    print("coarse model forward", flush=True)
    cfg, fe, ptr, idx, flags = coarse
    u, p, k, amp, dphi = _samples(cfg, fe, 5, 0)
    vec, par = _weights(cfg.m, 1, _scales(cfg, fe, u))
    s = _solver(cfg)
    assert s.coarse_n_params() == gnn.n_params(cfg.m)
    s.set_coarse_weights(vec)
    assert np.array_equal(s.get_coarse_weights(), vec)
    got = s.coarse_apply(k, u, p, amp, dphi)
    x = gnn.features(u, p, k, cfg.level_dt(1), cfg.m, fe, cfg.source, flags, par["scales"], amp, dphi)
    want, _ = gnn.forward(gnn.rounded(par), x, p, ptr, idx)
    corr_err = np.linalg.norm((got - p) - (want - p)) / np.linalg.norm(want - p)
    assert corr_err <= 1e-10, corr_err


def test_gradient_matches_oracle(coarse):
    """GPU gradients (FP32 accumulation) against the oracle's FP64 backward
    pass through the same bf16-rounded weights."""
    print("coarse model gradient", flush=True)
    cfg, fe, ptr, idx, flags = coarse
    u, p, k, amp, dphi = _samples(cfg, fe, 6, 2)
    vec, par = _weights(cfg.m, 3, _scales(cfg, fe, u))
    y = p + 0.04 * np.linalg.norm(u, axis=1, keepdims=True) / np.sqrt(fe.n) * \
        np.sin(np.arange(fe.n) * 0.01)[None]
    s = _solver(cfg)
    s.set_coarse_weights(vec)
    loss, g = s.coarse_gradient(k, u, p, y, amp, dphi)
    x = gnn.features(u, p, k, cfg.level_dt(1), cfg.m, fe, cfg.source, flags, par["scales"], amp, dphi)
    rp = gnn.rounded(par)
    psi, cache = gnn.forward(rp, x, p, ptr, idx)
    L, dpsi = gnn.loss(psi, y, par["scales"][2])
    gw = gnn.backward(rp, cache, dpsi, ptr, idx)
    assert abs(loss - L) <= 1e-5 * L
    gg = gnn.unpack(g.astype(np.float64), cfg.m)
    for name, _ in gnn.param_shapes(cfg.m):
        if name == "scales":
            assert np.all(gg[name] == 0)
            continue
        err = np.linalg.norm(gg[name] - gw[name]) / max(np.linalg.norm(gw[name]), 1e-30)
        assert err <= 2e-3, (name, err)


def test_adam_matches_oracle(coarse):
    print("coarse model adam", flush=True)
    cfg, fe, *_ = coarse
    vec, par = _weights(cfg.m, 4, [1.0, 1.0, 1.0, 0.0])
    rng = np.random.default_rng(5)
    g1 = rng.normal(size=vec.size).astype(np.float32)
    g2 = rng.normal(size=vec.size).astype(np.float32)
    g1[:4] = g2[:4] = 0
    s = _solver(cfg)
    s.set_coarse_weights(vec)
    s.coarse_adam(g1, 1e-2)
    s.coarse_adam(g2, 1e-2)
    got = s.get_coarse_weights().astype(np.float64)
    state = {}
    w = par
    for step, gv in enumerate((g1, g2), start=1):
        w = gnn.adam_step(w, gnn.unpack(gv.astype(np.float64), cfg.m), state, 1e-2, step)
    want = gnn.pack(w, cfg.m)
    assert np.max(np.abs(got - want)) <= 1e-5


def test_zero_output_layer_reproduces_implicit_euler(coarse):
    """delta = 0: the learned propagator is exactly the implicit-Euler step,
    so MGRIT runs the same iterations."""
    print("coarse model zero output", flush=True)
    cfg, fe, *_ = coarse
    vec, _ = _weights(cfg.m, 6, [1e-3, 1e5, 1e-4, 0.0], out_scale=0.0)
    ref = _solver(cfg)
    U0, st0 = ref.solve()
    s = _solver(cfg, coarse_model=1)
    s.set_coarse_weights(vec)
    U1, st1 = s.solve()
    assert st1["coarse_fallback"] == -1
    assert len(st1["rho"]) == len(st0["rho"])
    for a, b in zip(st1["rho"], st0["rho"]):
        assert abs(a - b) <= 1e-12 * st0["rho"][0]
    assert np.linalg.norm(U1 - U0) <= 1e-12 * np.linalg.norm(U0)


def test_untrained_random_network_still_converges(coarse):
    """Any coarse propagator keeps the fine fixed point (FAS); a poor one may
    be switched back to implicit Euler when the residual grows."""
    print("coarse model random", flush=True)
    cfg, fe, *_ = coarse
    H, _ = build(cfg)
    U_seq = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), cfg.n_steps)
    vec, _ = _weights(cfg.m, 7, [1e-3, 1e5, 2e-4, 0.0], out_scale=1.0)
    s = _solver(cfg, coarse_model=1)
    s.set_coarse_weights(vec)
    U, st = s.solve()
    assert st["converged"] and st["coarse_fallback"] == -1
    assert np.linalg.norm(U - U_seq) <= MGRIT_GATE * np.linalg.norm(U_seq)


def test_training_gain(coarse):
    """Trained on trajectories of the fine propagator with varied sources: the
    learned step is closer to m fine steps than implicit Euler on held-out
    trajectories (about 3.5x here), and MGRIT with it reaches the same solution
    without falling back to implicit Euler.  (Its MGRIT iteration count, 10
    against 8 here, is printed: the coarse correction depends on how the
    propagator maps errors, which trajectory pairs do not train.)"""
    print("coarse model training", flush=True)
    cfg, fe, *_ = coarse
    H, _ = build(cfg)
    U_seq = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), cfg.n_steps)
    s = _solver(cfg, coarse_model=1)
    ts = s.train_coarse(n_traj=64, epochs=8, batch=64, lr=2e-3, seed=11, perturb=0.3)
    print(ts, flush=True)
    assert ts["n_train"] > 0 and ts["n_val"] > 0
    assert ts["loss_last"] < 0.5 * ts["loss_first"]
    assert ts["val_err_learned"] < 0.5 * ts["val_err_ie"]
    U, st = s.solve()
    ref = _solver(cfg)
    _, st0 = ref.solve()
    print("iterations: learned", len(st["rho"]) - 1, "implicit Euler", len(st0["rho"]) - 1,
          "fallback", st["coarse_fallback"], flush=True)
    assert st["converged"] and st["coarse_fallback"] == -1
    assert np.linalg.norm(U - U_seq) <= MGRIT_GATE * np.linalg.norm(U_seq)
