"""Pins of the oracle's learned coarse propagator (network definition, manual
backward pass, Adam, bf16 rounding) against finite differences, closed forms
and adjoint identities."""

import math

import numpy as np
import pytest

from workload import polar_mesh, Source
from oracle.fe import MachineFE
from oracle.stepping import Level
from oracle import gnn


@pytest.fixture(scope="module")
def tiny():
    fe = MachineFE(polar_mesh(3, 8))        # 16 interior nodes on two rings
    ptr, idx = gnn.graph(fe)
    return fe, ptr, idx


def _random_params(m, seed, scale=0.4):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in gnn.param_shapes(m):
        p[name] = rng.uniform(-scale, scale, size=shape)
    p["scales"] = np.array([1.3, 0.7, 0.9, 0.0])
    return p


def test_ring_aggregation_closed_form():
    """One ring of interior nodes: the P1 neighbours are the two ring
    neighbours (the other vertices lie on the Dirichlet radii)."""
    fe = MachineFE(polar_mesh(2, 10))
    ptr, idx = gnn.graph(fe)
    assert np.all(np.diff(ptr) == 2)
    h = np.random.default_rng(0).normal(size=(10, 3))
    want = 0.5 * (np.roll(h, 1, axis=0) + np.roll(h, -1, axis=0))
    assert np.allclose(gnn.aggregate(ptr, idx, h), want, rtol=0, atol=1e-15)


def test_aggregation_adjoint(tiny):
    fe, ptr, idx = tiny
    rng = np.random.default_rng(1)
    h = rng.normal(size=(2, fe.n, 5))
    g = rng.normal(size=(2, fe.n, 5))
    lhs = np.sum(gnn.aggregate(ptr, idx, h) * g)
    rhs = np.sum(h * gnn.aggregate_t(ptr, idx, g))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_zero_output_layer_is_the_implicit_euler_step(tiny):
    fe, ptr, idx = tiny
    m = 2
    params = gnn.init_params(m, 0, [1.0, 1.0, 1.0, 0.0])
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, fe.n, gnn.n_features(m)))
    p = rng.normal(size=(3, fe.n))
    psi, _ = gnn.forward(params, x, p, ptr, idx)
    assert np.array_equal(psi, p)


def test_backward_matches_finite_differences(tiny):
    """Every parameter array: central differences of the loss agree with the
    manual backward pass (FP64, unrounded weights)."""
    fe, ptr, idx = tiny
    m = 2
    params = _random_params(m, 3)
    rng = np.random.default_rng(4)
    S = 2
    x = rng.normal(size=(S, fe.n, gnn.n_features(m)))
    p = rng.normal(size=(S, fe.n))
    y = rng.normal(size=(S, fe.n))

    def L(pr):
        psi, _ = gnn.forward(pr, x, p, ptr, idx)
        return gnn.loss(psi, y, pr["scales"][2])[0]

    psi, cache = gnn.forward(params, x, p, ptr, idx)
    _, dpsi = gnn.loss(psi, y, params["scales"][2])
    g = gnn.backward(params, cache, dpsi, ptr, idx)
    eps = 1e-6
    for name, shape in gnn.param_shapes(m):
        if name == "scales":
            continue
        flat = params[name].ravel()
        picks = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for k in picks:
            pp = {kk: v.copy() for kk, v in params.items()}
            pm = {kk: v.copy() for kk, v in params.items()}
            pp[name].ravel()[k] += eps
            pm[name].ravel()[k] -= eps
            fd = (L(pp) - L(pm)) / (2 * eps)
            an = g[name].ravel()[k]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)), (name, k, fd, an)


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    psi = rng.normal(size=(2, 7))
    y = rng.normal(size=(2, 7))
    L0, d = gnn.loss(psi, y, 0.6)
    e = np.zeros_like(psi)
    e[1, 3] = 1e-6
    fd = (gnn.loss(psi + e, y, 0.6)[0] - gnn.loss(psi - e, y, 0.6)[0]) / 2e-6
    assert abs(fd - d[1, 3]) <= 1e-8
    assert abs(L0 - np.mean(((psi - y) / 0.6) ** 2)) <= 1e-15


def test_bf16_rounding_hand_values():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, math.pi, -2.5, 1.0 + 2.0 ** -7 + 2.0 ** -8])
    want = [1.0, 1.0, 1.0 + 2.0 ** -7, 3.140625, -2.5, 1.0 + 2.0 ** -6]
    assert np.array_equal(gnn.bf16_round(v), want)


def test_adam_first_step_is_a_signed_step():
    """From zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    w = {"scales": np.zeros(4), "a": np.array([0.5, -1.0, 2.0])}
    g = {"scales": np.zeros(4), "a": np.array([0.3, -4.0, 1e-3])}
    out = gnn.adam_step(w, g, {}, lr=0.01, step=1)
    want = w["a"] - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8)
    assert np.allclose(out["a"], want, rtol=1e-12, atol=0)
    assert np.array_equal(out["scales"], w["scales"])


def test_source_features_are_the_forcing_of_the_shifted_source():
    fe = MachineFE(polar_mesh(4, 32))
    src = Source(ramp_periods=2.0)
    flags = gnn.node_flags(fe)
    m, dT = 4, 2.5e-4
    k = np.array([3, 17])
    amp, dphi = np.array([1.2, 0.85]), np.array([0.3, -1.1])
    x = gnn.features(np.zeros((2, fe.n)), np.zeros((2, fe.n)), k, dT, m, fe, src, flags,
                     [1.0, 2.0e4, 1.0, 0.0], amp, dphi)
    for s in range(2):
        from dataclasses import replace
        lev = Level(fe.mesh, 1e-4, replace(src, amplitude=amp[s], phase_offset=dphi[s]), fe=fe)
        t = k[s] * dT + np.arange(m + 1) * dT / m
        assert np.allclose(x[s, :, 2:m + 3], lev.forcing(t).T / 2.0e4, rtol=1e-14, atol=0)
    assert np.array_equal(x[0, :, m + 3:], flags)
    assert flags[:, 3].min() > 0 and flags[:, 3].max() < 1


def test_adam_training_reduces_the_loss(tiny):
    fe, ptr, idx = tiny
    m = 2
    rng = np.random.default_rng(6)
    x = rng.normal(size=(4, fe.n, gnn.n_features(m)))
    p = rng.normal(size=(4, fe.n))
    y = p + 0.3 * np.tanh(x[..., 0])        # a learnable correction
    params = gnn.init_params(m, 1, [1.0, 1.0, 1.0, 0.0])
    state = {}
    losses = []
    for step in range(1, 41):
        psi, cache = gnn.forward(params, x, p, ptr, idx)
        L, d = gnn.loss(psi, y, 1.0)
        losses.append(L)
        params = gnn.adam_step(params, gnn.backward(params, cache, d, ptr, idx), state, 0.01, step)
    assert losses[-1] < 0.2 * losses[0]


def test_parameter_count_and_layout():
    m = 16
    assert gnn.n_features(m) == 23
    assert gnn.n_params(m) == 4 + 23 * 64 + 64 + 3 * (2 * 64 * 64 + 64) + 64 + 1
    v = np.arange(gnn.n_params(m), dtype=np.float64)
    assert np.array_equal(gnn.pack(gnn.unpack(v, m), m), v)


def test_node_flags_from_the_band_layout():
    """Node flags of the 16 x 128 machine mesh derived independently of the
    finite-element matrices: every radial cell row of 5 mm belongs to one band
    of the layout (rows 0-4 rotor iron, 5-6 bar band, 7 air gap, 8-10 slot
    band, 11-15 stator iron); in the bar band a cell is an aluminium bar when
    its centre angle lies in the first half of a 1/28 pitch, in the slot band
    a coil when it lies in the first half of a 1/36 pitch (integer tests on
    (2j+1) * pitches mod 256, exact); interior node (i, j) touches the cells
    (i-1, j-1), (i-1, j), (i, j-1), (i, j).  Flags: conductor, iron, coil,
    normalised radius i/16."""
    n_r, n_t = 16, 128
    fe = MachineFE(polar_mesh(n_r, n_t))
    got = gnn.node_flags(fe)
    assert got.shape == ((n_r - 1) * n_t, 4)

    def cell(i, j):
        j %= n_t
        bar = ((2 * j + 1) * 28) % 256 < 128
        slot = ((2 * j + 1) * 36) % 256 < 128
        if i <= 4:
            return "iron"
        if i <= 6:
            return "bar" if bar else "iron"
        if i == 7:
            return "air"
        if i <= 10:
            return "coil" if slot else "iron"
        return "iron"

    want = np.zeros_like(got)
    for i in range(1, n_r):
        for j in range(n_t):
            kinds = {cell(i - 1, j - 1), cell(i - 1, j), cell(i, j - 1), cell(i, j)}
            k = (i - 1) * n_t + j
            want[k] = ["bar" in kinds, "iron" in kinds, "coil" in kinds, i / n_r]
    assert np.array_equal(got[:, :3], want[:, :3])
    assert np.allclose(got[:, 3], want[:, 3], rtol=0, atol=1e-12)
    # hand-checked nodes: (1, 0) rotor iron only; (6, 0) bar cell (5, 0) next
    # to iron cell (5, 127); (8, 0) slot cell (8, 0) next to the tooth (8, 127)
    assert list(got[0, :3]) == [0, 1, 0]
    assert list(got[5 * n_t, :3]) == [1, 1, 0]
    assert list(got[7 * n_t, :3]) == [0, 1, 1]
    # ring 7 touches only the bar band and the air gap: no coil there
    assert not got[6 * n_t:7 * n_t, 2].any()
