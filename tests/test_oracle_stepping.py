"""Pins of the oracle's propagator and sequential solve (Sec. 2, eq. 2 and the
space-time block system; Sec. 3.1, eq. 8) against brute force and textbook
special cases."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workload import polar_mesh, Source, BHLaw
from oracle.stepping import Level, sequential
from oracle.fe import MachineFE
from oracle import pwm


@pytest.fixture(scope="module")
def tiny():
    mesh = polar_mesh(4, 16)
    return Level(mesh, 0.02 / 32, Source())


def test_space_time_brute_force(tiny):
    """Assemble the whole block lower-bidiagonal system (implicit Euler written
    as one sparse matrix over all 33 time points) and solve it with one sparse
    LU: it must equal the sequential forward block solve."""
    L, N = tiny, 32
    n = L.n
    Mdt = L.fe.M / L.dt
    A = (Mdt + L.fe.K).tocsr()
    blocks = [[None] * (N + 1) for _ in range(N + 1)]
    blocks[0][0] = sp.identity(n)
    for i in range(1, N + 1):
        blocks[i][i] = A
        blocks[i][i - 1] = -Mdt
    big = sp.bmat(blocks, format="csc")
    rhs = np.zeros((N + 1, n))
    rhs[1:] = L.forcing(np.arange(1, N + 1) * L.dt)
    U_bf = spla.spsolve(big, rhs.ravel()).reshape(N + 1, n)
    U_seq = sequential(L, np.zeros(n), N)
    assert np.linalg.norm(U_seq - U_bf) <= 1e-10 * np.linalg.norm(U_bf)  # big LU of a badly scaled block system
    assert np.linalg.norm(U_bf) > 0


def test_phi_dense_inverse(tiny):
    """Phi(u) = (M/dt + K)^{-1} ((M/dt) u + f(t_{i+1})) with a dense inverse."""
    L = tiny
    rng = np.random.default_rng(0)
    u = rng.standard_normal((3, L.n)) * 1e-3
    i_from = np.array([0, 7, 31])
    A = (L.fe.M.toarray() / L.dt + L.fe.K.toarray())
    Ainv = np.linalg.inv(A)
    t = (i_from + 1) * L.dt
    b = pwm.phase_signals(t, L.source).T @ L.fe.F * L.source.J0
    ref = (Ainv @ ((L.fe.M.toarray() / L.dt) @ u.T + b.T)).T
    got = L.phi(u, i_from)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_zero_conductivity_is_magnetostatic():
    """Where sigma = 0 everywhere, Phi forgets u_prev: K u = f(t)."""
    mesh = polar_mesh(4, 16)
    fe = MachineFE(mesh)
    fe.M = fe.M * 0.0
    L = Level(mesh, 1e-5, Source(), fe=fe)
    u1 = L.phi(np.ones((1, L.n)), [3])[0]
    u2 = L.phi(np.zeros((1, L.n)), [3])[0]
    assert np.allclose(u1, u2, rtol=0, atol=1e-15)
    ref = spla.spsolve(fe.K.tocsc(), L.forcing(np.array([4e-5]))[0])
    assert np.linalg.norm(u1 - ref) <= 1e-12 * np.linalg.norm(ref)


def test_newton_linear_limit_one_iteration():
    """k1 = 0 makes nu = k3 constant in iron: Newton converges in one step and
    equals the linear solve with mu_r = 1 / (mu0 k3)."""
    mesh = polar_mesh(4, 32)
    bh = BHLaw(nonlinear=True, k1=0.0, k3=500.0)
    Ln = Level(mesh, 1e-5, Source(), bh=bh)
    fe_lin = MachineFE(mesh)
    fe_lin.nu_cell = np.where(fe_lin.iron_cell, 500.0, fe_lin.nu_cell)
    from oracle.fe import stiffness
    K = stiffness(mesh.xy, mesh.tri, fe_lin.nu_cell)
    fe_lin.K = K[fe_lin.free][:, fe_lin.free].tocsr()
    Ll = Level(mesh, 1e-5, Source(), fe=fe_lin)
    u0 = np.zeros((1, Ln.n))
    un = Ln.phi(u0, [10])[0]
    ul = Ll.phi(u0, [10])[0]
    assert Ln.newton_iters[-1] == 1
    assert np.linalg.norm(un - ul) <= 1e-12 * np.linalg.norm(ul)


def test_newton_jacobian_matches_finite_differences():
    mesh = polar_mesh(4, 32)
    bh = BHLaw(nonlinear=True)
    L = Level(mesh, 1e-5, Source(), bh=bh)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(L.n) * 5e-3        # |B| ~ 1 T in iron
    f = np.zeros(L.n)
    J = (L.Mdt + L.fe.jacobian_nonlinear(u, bh)).toarray()
    h = 1e-7 * np.abs(u).max()
    cols = rng.choice(L.n, 12, replace=False)
    for c in cols:
        e = np.zeros(L.n)
        e[c] = h
        fd = (L.residual(u + e, u, f) - L.residual(u - e, u, f)) / (2 * h)
        assert np.linalg.norm(fd - J[:, c]) <= 1e-6 * np.linalg.norm(J[:, c])


def test_newton_solution_satisfies_residual():
    """A source strong enough to saturate the iron (|B| ~ 2 T): Newton needs
    several iterations and its result zeroes the residual."""
    mesh = polar_mesh(4, 32)
    bh = BHLaw(nonlinear=True)
    L = Level(mesh, 1e-5, Source(J0=4e7), bh=bh)
    u_prev = np.zeros(L.n)
    u = L.phi(u_prev[None], [3])[0]
    f = L.forcing(np.array([4e-5]))[0]
    r0 = np.linalg.norm(L.residual(u_prev, u_prev, f))
    assert np.linalg.norm(L.residual(u, u_prev, f)) <= 1e-10 * r0
    assert L.newton_iters[-1] >= 3
    nu, _ = L.fe.nu_nonlinear(L.fe.b_squared(u), bh)
    assert np.ptp(nu[L.fe.iron_cell]) > 100.0


def test_damped_newton_reaches_the_root_plain_newton_misses():
    """Damped Newton (Sec. 5.1; Armijo step lengths): at a source so strong
    that a full Newton step from u = 0 overflows the reluctivity, plain Newton
    fails while the damped iteration takes shortened steps and ends at a zero
    of the residual."""
    mesh = polar_mesh(8, 64)
    bh = BHLaw(nonlinear=True)
    plain = Level(mesh, 1e-4, Source(J0=3e8), bh=bh, newton_maxit=30, newton_halvings=0)
    with pytest.raises(Exception):
        plain.phi(np.zeros((1, plain.n)), [3])
    L = Level(mesh, 1e-4, Source(J0=3e8), bh=bh, newton_maxit=30, newton_halvings=6)
    u = L.phi(np.zeros((1, L.n)), [3])[0]
    assert min(L.newton_lambdas) < 1.0
    f = L.forcing(np.array([4e-4]))[0]
    r0 = np.linalg.norm(L.residual(np.zeros(L.n), np.zeros(L.n), f))
    assert np.linalg.norm(L.residual(u, np.zeros(L.n), f)) <= 1e-10 * r0


def test_damping_does_not_move_the_root():
    """Where plain Newton converges, damped Newton lands on the same solution."""
    mesh = polar_mesh(8, 64)
    bh = BHLaw(nonlinear=True)
    out = []
    for hv in (0, 6):
        L = Level(mesh, 1e-4, Source(J0=1e8), bh=bh, newton_maxit=30, newton_halvings=hv)
        out.append(L.phi(np.zeros((1, L.n)), [3])[0])
        if hv:
            assert min(L.newton_lambdas) < 1.0
    assert np.linalg.norm(out[0] - out[1]) <= 1e-9 * np.linalg.norm(out[0])


def test_window_with_shifted_time_origin_continues_the_trajectory():
    """A run of 48 steps whose source starts at t_start = 200 dt, started
    from the state at step 200, continues the 248-step trajectory."""
    from dataclasses import replace
    from workload import config
    cfg = config("cfg1")
    mesh = polar_mesh(16, 128)
    lev = Level(mesh, cfg.dt, cfg.source)
    U = sequential(lev, np.zeros(lev.n), 248)
    win = Level(mesh, cfg.dt, replace(cfg.source, t_start=200 * cfg.dt))
    W = sequential(win, U[200], 48)
    assert np.linalg.norm(W - U[200:]) <= 1e-12 * np.linalg.norm(U[200:])
