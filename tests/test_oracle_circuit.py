"""Pins of the oracle's field-circuit coupled step (Sec. 3.1, the stator coil
and rotor bar circuit equations) against facts outside it: Kirchhoff's laws
on the full two-ring cage network, the textbook RL circuit of a winding
without conductors, the discrete energy balance of backward Euler, and the
sequential solution and finite termination of MGRIT (Algorithm 1)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workload import polar_mesh, Source, Circuit, config
from oracle.circuit import CircuitLevel, cage_matrix
from oracle.fe import MachineFE
from oracle.problem import build
from oracle import mgrit, stepping


def test_cage_matrix_matches_nodal_analysis():
    """Two end rings (ring_r between neighbouring nodes), bar k between node
    k of ring 1 and node k of ring 2 carrying i_k = G_k v_k - e_k: Kirchhoff's
    current law at every node, solved for the node potentials (one node
    grounded), gives bar voltages v with cage_matrix(G, ring_r) v = e."""
    rng = np.random.default_rng(3)
    for nb in (3, 7, 28):
        G = rng.uniform(1.0, 5.0, nb)
        e = rng.standard_normal(nb)
        ring_r = rng.uniform(0.05, 2.0)
        # unknowns: phi1[0..nb-1], phi2[0..nb-1]; phi2[0] = 0 replaces its KCL row
        N = 2 * nb
        A = np.zeros((N, N))
        b = np.zeros(N)
        g = 1.0 / ring_r
        for k in range(nb):
            r1, r2 = k, nb + k
            # ring 1, node k: current into bar k plus currents into both ring segments = 0
            A[r1, r1] += G[k]
            A[r1, r2] -= G[k]
            b[r1] += e[k]
            # ring 2, node k: current out of bar k is the current arriving
            A[r2, r2] += G[k]
            A[r2, r1] -= G[k]
            b[r2] -= e[k]
            for j in ((k + 1) % nb, (k - 1) % nb):
                A[r1, r1] += g
                A[r1, j] -= g
                A[r2, r2] += g
                A[r2, nb + j] -= g
        A[nb] = 0.0
        A[nb, nb] = 1.0
        b[nb] = 0.0
        phi = np.linalg.solve(A, b)
        v = phi[:nb] - phi[nb:]
        assert np.allclose(cage_matrix(G, ring_r) @ v, e, rtol=1e-12, atol=1e-12)
        # the rings carry the bars' currents back: they sum to zero
        i = G * v - e
        assert abs(i.sum()) <= 1e-12 * np.abs(i).max()


def test_winding_without_conductors_is_an_rl_circuit():
    """With sigma = 0 everywhere and no rotor circuit, a_i = K^{-1} X^T i1_i
    and the coil equations reduce to the backward-Euler RL circuit
    (L/dt + R) i_i = v(t_i) + (L/dt) i_{i-1} with the inductance matrix
    L = l_z X K^{-1} X^T (computed here densely)."""
    mesh = polar_mesh(6, 24)
    fe = MachineFE(mesh)
    fe.M = 0.0 * fe.M
    fe.sigma_cell = 0.0 * fe.sigma_cell
    circ = Circuit(rotor=False, r_phase=0.8)
    dt = 0.02 / 256
    lev = CircuitLevel(mesh, dt, Source(), circ, fe=fe)
    K = fe.K.toarray()
    KX = np.linalg.solve(K, lev.X.T)                       # [n, 3]
    Lm = circ.l_z * lev.X @ KX
    a = np.zeros(lev.n)
    i_prev = np.zeros(3)
    for i in range(40):
        a, i1, v2 = lev.step(a[None], [i])
        a, i1 = a[0], i1[0]
        v = lev.voltages([(i + 1) * dt])[0]
        i_rl = np.linalg.solve(Lm / dt + circ.r_phase * np.eye(3), v + Lm @ i_prev / dt)
        assert np.allclose(i1, i_rl, rtol=1e-9, atol=1e-9 * np.abs(i_rl).max())
        assert np.linalg.norm(a - KX @ i_rl) <= 1e-9 * np.linalg.norm(a)
        assert v2.shape == (1, 0)
        i_prev = i_rl
    assert np.abs(i_prev).max() > 0.0


def test_energy_balance_of_every_step():
    """Multiplying the field rows by l_z (a_i - a_{i-1})^T and using the
    circuit rows: per step
      (l_z/dt) |a_i - a_{i-1}|_M^2 + l_z (a_i - a_{i-1})^T K a_i
        = dt (v . i1 - R |i1|^2) + dt v2^T C v2,
    an identity of the coupled backward-Euler step (a wrong sign or factor in
    any coupling term breaks it)."""
    cfg = config("cfg1", circuit=Circuit())
    H, _ = build(cfg)
    lev = H.levels[0]
    c = cfg.circuit
    dt = lev.dt
    M, K = lev.fe.M, lev.fe.K
    a = np.zeros(lev.n)
    for i in range(60):
        a_new, i1, v2 = lev.step(a[None], [i])
        a_new, i1, v2 = a_new[0], i1[0], v2[0]
        d = a_new - a
        left = c.l_z / dt * d @ (M @ d) + c.l_z * d @ (K @ a_new)
        v = lev.voltages([(i + 1) * dt])[0]
        right = dt * (v @ i1 - c.r_phase * i1 @ i1) + dt * v2 @ lev.C @ v2
        scale = abs(c.l_z / dt * d @ (M @ d)) + abs(c.l_z * d @ (K @ a_new)) + dt * abs(v @ i1)
        assert abs(left - right) <= 1e-9 * scale, (i, left, right)
        a = a_new
    assert np.abs(v2).max() > 0.0 and np.abs(i1).max() > 0.0


def test_circuit_values_reproduce_the_coupled_solve():
    """The currents and voltages recovered from two consecutive states by the
    circuit rows alone equal the bordered solve's."""
    cfg = config("cfg1", circuit=Circuit())
    H, _ = build(cfg)
    lev = H.levels[0]
    U = stepping.sequential(lev, np.zeros(lev.n), 40)
    _, i1, v2 = lev.step(U[:-1], np.arange(40))
    j1, w2, j2 = lev.circuit_values(U[:-1], U[1:], np.arange(40))
    assert np.allclose(j1, i1, rtol=1e-8, atol=1e-8 * np.abs(i1).max())
    assert np.allclose(w2, v2, rtol=1e-8, atol=1e-8 * np.abs(v2).max())
    # Kirchhoff: the bar currents return through the rings
    assert np.abs(j2.sum(axis=1)).max() <= 1e-9 * np.abs(j2).max()


def test_mgrit_with_circuit_reaches_the_sequential_solution():
    """FAS-MGRIT with the coupled propagator on two levels: FCF relaxation is
    exact after N_t / (2m) iterations (the exactness front of Algorithm 1),
    and the tolerance-driven solve matches sequential stepping."""
    cfg = config("cfg1", n_steps=128, t_final=128 * 0.02 / 1024, m=4, circuit=Circuit())
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    U, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=0.0, maxit=cfg.n_steps // (2 * cfg.m))
    assert np.linalg.norm(U - U_seq) <= 1e-11 * np.linalg.norm(U_seq)
    U, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=1e-9, maxit=40)
    assert hist[-1] <= 1e-9 * hist[0]
    assert np.linalg.norm(U - U_seq) <= 1e-7 * np.linalg.norm(U_seq)
    assert len(hist) - 1 < cfg.n_steps // (2 * cfg.m)


def test_nonlinear_circuit_is_rejected():
    cfg = config("cfg4", circuit=Circuit())
    with pytest.raises(NotImplementedError):
        build(cfg)
