"""Pins of the oracle's F-cycles, nested iteration and Joule losses
(Sec. 2.1 cycles and nested iteration, Sec. 3.1 loss integral, Sec. 5.1 stop
rule) against facts that do not come from the oracle's own step loops:

  * the textbook level-visit order of an F-cycle on four levels (Fig. 4);
  * F-cycles on two levels are V-cycles;
  * finite termination after N_t / (2m) FCF iterations without spatial
    coarsening (Sec. 2.1) also holds for F-cycles;
  * the whole iteration written as block solves of the dense space-time
    matrices (no time-stepping loop) gives the same residual histories and
    iterates for V-cycles, F-cycles and the nested-iteration start, with and
    without spatial coarsening;
  * nested iteration with the ideal coarse propagator reproduces sequential
    stepping exactly;
  * the loss of a field uniform in space and linear in time is
    a^2 * sum(sigma * area) (consistent mass reproduces constants).
"""

from dataclasses import replace

import numpy as np
import pytest

from workload import config, polar_mesh, Source
from workload.configs import LevelSpec
from oracle.problem import build
from oracle import mgrit, stepping


def _tiny_cfg(meshes, n_steps, m, **kw):
    cfg = config("cfg1", meshes=[LevelSpec(*mm) for mm in meshes], n_steps=n_steps,
                 t_final=n_steps * 0.02 / 1024, **kw)
    cfg.m = m
    return cfg


def _compress(seq):
    out = []
    for v in seq:
        if not out or out[-1] != v:
            out.append(v)
    return out


def test_f_cycle_visits_levels_in_the_textbook_order():
    cfg = _tiny_cfg([(4, 16)] * 4, 32, 2)
    H, _ = build(cfg)
    H.cycle = "F"
    mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, maxit=1)
    assert _compress(H.visits) == [0, 1, 2, 3, 2, 3, 2, 1, 2, 3, 2, 1, 0]
    H.visits = []
    H.cycle = "V"
    mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, maxit=1)
    assert _compress(H.visits) == [0, 1, 2, 3, 2, 1, 0]


def test_two_level_f_cycle_is_the_v_cycle():
    cfg = _tiny_cfg([(4, 16), (4, 16)], 64, 4)
    out = []
    for kind in ("V", "F"):
        H, _ = build(cfg)
        H.cycle = kind
        out.append(mgrit.solve(H, np.zeros(H.levels[0].n), cfg.n_steps, maxit=6))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


def test_f_cycle_exact_after_nt_over_2m_fcf():
    cfg = _tiny_cfg([(4, 16)] * 3, 64, 4)
    H, _ = build(cfg)
    H.cycle = "F"
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    U, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=0.0, maxit=cfg.n_steps // (2 * cfg.m))
    assert np.linalg.norm(U - U_seq) <= 1e-12 * np.linalg.norm(U_seq)


# --- the iteration as block solves of dense space-time matrices -------------

class DenseLevel:
    """Level l of a linear hierarchy as one dense space-time system
    A_st u = g + c: A_st = I with -Phi on the block subdiagonal, c_i the
    forcing part of step i (Phi(u) = Phi_lin u + c_{i+1})."""

    def __init__(self, lev, N):
        n = lev.n
        A = (lev.Mdt + lev.fe.K).toarray()
        Phi = np.linalg.solve(A, lev.Mdt.toarray())
        t = np.arange(1, N + 1) * lev.dt
        c = np.zeros((N + 1, n))
        c[1:] = np.linalg.solve(A, lev.forcing(t).T).T
        S = np.zeros(((N + 1) * n, (N + 1) * n))
        for i in range(1, N + 1):
            S[i * n:(i + 1) * n, (i - 1) * n:i * n] = Phi
        self.n, self.N = n, N
        self.A = np.eye((N + 1) * n) - S
        self.c = c

    def op(self, u):
        """The FAS operator A(u): u_0, u_i - Phi(u_{i-1})."""
        return (self.A @ u.ravel()).reshape(u.shape) - self.c


class DenseHierarchy:
    def __init__(self, H, n_steps):
        self.H = H
        self.L = len(H.levels)
        Ns = [n_steps]
        for l in range(self.L - 1):
            Ns.append(Ns[-1] // H.ms[l])
        self.lev = [DenseLevel(H.levels[l], Ns[l]) for l in range(self.L)]

    def _masks(self, l):
        N = self.lev[l].N
        pts = np.arange(N + 1)
        m = self.H.ms[l] if l < self.L - 1 else 1
        return pts % m == 0, pts % m != 0

    def _rows(self, l, mask):
        n = self.lev[l].n
        return (np.nonzero(mask)[0][:, None] * n + np.arange(n)[None, :]).ravel()

    def f_relax(self, l, u, g):
        D = self.lev[l]
        C, F = self._masks(l)
        rf, rc = self._rows(l, F), self._rows(l, C)
        rhs = (g + D.c).ravel()
        x = u.ravel().copy()
        x[rf] = np.linalg.solve(D.A[np.ix_(rf, rf)], rhs[rf] - D.A[np.ix_(rf, rc)] @ x[rc])
        u[:] = x.reshape(u.shape)

    def c_relax(self, l, u, g):
        D = self.lev[l]
        C, F = self._masks(l)
        rf, rc = self._rows(l, F), self._rows(l, C)
        rhs = (g + D.c).ravel()
        x = u.ravel().copy()
        x[rc] = rhs[rc] - D.A[np.ix_(rc, rf)] @ x[rf]
        u[:] = x.reshape(u.shape)

    def relax(self, l, u, g):
        self.f_relax(l, u, g)
        for _ in range(self.H.gamma):
            self.c_relax(l, u, g)
            self.f_relax(l, u, g)

    def residual(self, l, u, g):
        C, _ = self._masks(l)
        return (g - self.lev[l].op(u))[C]

    def coarse_correct(self, l, u, g, r, kind):
        R, P = self.H.R[l], self.H.P[l]
        tr = (lambda T, x: x.copy()) if R is None else (lambda T, x: (T @ x.T).T)
        C, _ = self._masks(l)
        u2 = tr(R, u[C])
        g2 = self.lev[l + 1].op(u2) + tr(R, r)
        v = u2.copy()
        if kind == "F":
            self.cycle(l + 1, v, g2, "F")
            if l + 1 < self.L - 1:
                self.cycle(l + 1, v, g2, "V")
        else:
            self.cycle(l + 1, v, g2, "V")
        u[C] += tr(P, v - u2)

    def cycle(self, l, u, g, kind):
        D = self.lev[l]
        if l == self.L - 1:
            u[:] = np.linalg.solve(D.A, (g + D.c).ravel()).reshape(u.shape)
            return
        self.relax(l, u, g)
        r = self.residual(l, u, g)
        self.coarse_correct(l, u, g, r, kind)
        self.f_relax(l, u, g)

    def solve(self, iters, kind, guess=None):
        D = self.lev[0]
        u = np.zeros((D.N + 1, D.n)) if guess is None else guess.copy()
        g = np.zeros_like(u)
        hist = []
        for it in range(iters + 1):
            self.relax(0, u, g)
            hist.append(float(np.linalg.norm(self.residual(0, u, g))))
            if it < iters:
                self.coarse_correct(0, u, g, self.residual(0, u, g), kind)
        return u, hist

    def nested(self):
        uc = None
        for l in range(self.L - 1, -1, -1):
            D = self.lev[l]
            u = np.zeros((D.N + 1, D.n))
            g = np.zeros_like(u)
            if l == self.L - 1:
                u[:] = np.linalg.solve(D.A, (g + D.c).ravel()).reshape(u.shape)
            else:
                P = self.H.P[l]
                u[::self.H.ms[l]] = uc if P is None else (P @ uc.T).T
                self.cycle(l, u, g, "V")
            uc = u
        return uc


# with spatial coarsening the coarse mesh 4 x 16 still carries coil cells
# (its ring of cells at r = 0.06-0.08 m lies in the slot band)
MESHES = {"no_sc": ([(4, 16)] * 3, 32), "sc": ([(8, 32), (4, 16), (4, 16)], 16)}


@pytest.mark.parametrize("case", ["no_sc", "sc"])
@pytest.mark.parametrize("kind", ["V", "F"])
def test_cycles_match_dense_space_time_block_solves(case, kind):
    meshes, N = MESHES[case]
    cfg = _tiny_cfg(meshes, N, 2)
    H, _ = build(cfg)
    H.cycle = kind
    n = H.levels[0].n
    U, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=0.0, maxit=3)
    D = DenseHierarchy(H, cfg.n_steps)
    Ud, hd = D.solve(3, kind)
    for a, b in zip(hist, hd):
        assert abs(a - b) <= 1e-10 * hd[0], (a, b)
    assert np.linalg.norm(U - Ud) <= 1e-10 * np.linalg.norm(Ud)


@pytest.mark.parametrize("case", ["no_sc", "sc"])
def test_nested_iteration_matches_dense_space_time_block_solves(case):
    meshes, N = MESHES[case]
    cfg = _tiny_cfg(meshes, N, 2, source=Source(signal="sine"))
    H, _ = build(cfg)
    n = H.levels[0].n
    G = mgrit.nested_iteration(H, np.zeros(n), cfg.n_steps)
    Gd = DenseHierarchy(H, cfg.n_steps).nested()
    assert np.linalg.norm(G - Gd) <= 1e-10 * np.linalg.norm(Gd)


def test_nested_iteration_with_the_ideal_coarse_propagator_is_exact():
    """Two levels, coarse propagator = m fine steps, one source: the coarsest
    sequential solve gives the exact C-point values, the finest V-cycle's
    relaxation the exact F-points."""
    cfg = _tiny_cfg([(4, 16), (4, 16)], 64, 4)
    H, _ = build(cfg)
    H.levels[1] = mgrit.ExactCoarse(H.levels[0], cfg.m)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    G = mgrit.nested_iteration(H, np.zeros(n), cfg.n_steps)
    assert np.linalg.norm(G - U_seq) <= 1e-12 * np.linalg.norm(U_seq)


def test_sine_source_is_the_reference_signal():
    """signal = "sine": the coil currents follow the three sine references."""
    from oracle import pwm
    src = Source(signal="sine")
    t = np.linspace(0.0, 0.02, 17)
    b = pwm.phase_signals(t, src)
    for p in range(3):
        assert np.allclose(b[p], np.sin(2 * np.pi * 50.0 * t + src.phases[p]), atol=1e-15)


def test_nested_iteration_start_is_closer_than_zero():
    """On the PWM problem the sine-driven nested-iteration start leaves a
    smaller first C-point residual than the zero start (Sec. 4.1 uses it as
    an improved initial guess)."""
    cfg = _tiny_cfg([(8, 32)] * 3, 256, 4)
    H, _ = build(cfg)
    Hs, _ = build(replace(cfg, source=Source(signal="sine")))
    n = H.levels[0].n
    guess = mgrit.nested_iteration(Hs, np.zeros(n), cfg.n_steps)
    _, h0, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, maxit=0)
    _, h1, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, maxit=0, guess=guess)
    assert h1[0] < 0.5 * h0[0], (h0, h1)


def test_joule_loss_of_a_uniform_linear_ramp():
    """u_i = a t_i on every unknown: du/dt = a everywhere in the interior, and
    the consistent sigma-mass matrix integrates the constant exactly over
    the bars, except the boundary rings whose nodes are fixed to 0 do not
    touch any bar, so P = a^2 * sum over bar cells of sigma * area."""
    from oracle.fe import MachineFE
    from workload.machine import material_arrays
    mesh = polar_mesh(16, 128)
    fe = MachineFE(mesh)
    lev = stepping.Level(mesh, 1e-5, Source())
    _, sigma, _ = material_arrays()
    xy = mesh.xy[mesh.tri]
    area = 0.5 * np.abs((xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1]) -
                        (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1]))
    want_unit = float(np.sum(sigma[mesh.cell_mat] * area))
    a, dt = 3.0, 1e-5
    u_prev = np.full(fe.n, a * 4 * dt)
    u = np.full(fe.n, a * 5 * dt)
    p = mgrit.joule_losses(lev, u_prev, u, dt)
    assert abs(p[0] - a * a * want_unit) <= 1e-12 * a * a * want_unit
    # zero change, zero loss; scaling the change by s scales the loss by s^2
    assert mgrit.joule_losses(lev, u, u, dt)[0] == 0.0
    p2 = mgrit.joule_losses(lev, u_prev, u_prev + 2.0 * (u - u_prev), dt)[0]
    assert abs(p2 - 4.0 * p[0]) <= 1e-12 * p2


def test_max_relative_change_hand_values():
    assert mgrit.max_relative_change([1.0, 2.0, 0.0], [1.01, 2.0, 0.0]) == pytest.approx(0.01)
    assert mgrit.max_relative_change([0.0, 0.0], [0.0, 0.0]) == 0.0
    assert mgrit.max_relative_change([4.0, 1.0], [3.0, 1.0]) == pytest.approx(0.25)


def test_loss_stop_rule_ends_when_the_losses_settle():
    """Sec. 5.1: stop once no C-point loss changes by 1 % or more between two
    iterations.  The stopping iterate's losses are then within a few percent
    of those of sequential stepping, and a tighter threshold takes at least
    as many iterations."""
    cfg = _tiny_cfg([(8, 32)] * 3, 256, 4)
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    its = []
    for tol in (1e-2, 1e-4):
        losses = []
        H.visits = []
        U, hist, conv = mgrit.solve(H, np.zeros(n), cfg.n_steps, maxit=40, loss_tol=tol, losses=losses)
        assert conv
        assert mgrit.max_relative_change(losses[-1], losses[-2]) < tol
        its.append(len(hist))
        p_seq = mgrit.c_point_losses(H, U_seq)
        nz = p_seq > 1e-6 * p_seq.max()
        rel = np.abs(losses[-1][nz] - p_seq[nz]) / p_seq[nz]
        assert rel.max() < 20 * tol, rel.max()
    assert its[1] >= its[0]


# --- per-level coarsening factors and delayed spatial coarsening -------------

def test_per_level_factors_match_dense_space_time_block_solves():
    """Four levels with m = 4 on the first level and 2 below (the paper's
    pattern of a large first factor and small coarse ones, Sec. 4.1), with
    spatial coarsening on the last level: V- and F-cycles against the dense
    block solves."""
    cfg = _tiny_cfg([(8, 32), (8, 32), (8, 32), (4, 16)], 16, 4, m_coarse=2)
    assert cfg.level_factors() == [4, 2, 2] and cfg.level_steps(3) == 1
    for kind in ("V", "F"):
        H, _ = build(cfg)
        H.cycle = kind
        n = H.levels[0].n
        U, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=0.0, maxit=2)
        Ud, hd = DenseHierarchy(H, cfg.n_steps).solve(2, kind)
        for a, b in zip(hist, hd):
            assert abs(a - b) <= 1e-10 * hd[0], (kind, a, b)
        assert np.linalg.norm(U - Ud) <= 1e-10 * np.linalg.norm(Ud)


def test_five_level_exact_after_nt_over_2m0_fcf():
    """Five levels, m = 4 then 2, no spatial coarsening: FCF relaxation on the
    finest level makes two more of its intervals exact per iteration, so the
    iterate is the sequential solution after N_t / (2 m_0) iterations."""
    cfg = _tiny_cfg([(4, 16)] * 5, 128, 4, m_coarse=2)
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    U, _, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=0.0, maxit=cfg.n_steps // (2 * cfg.m))
    assert np.linalg.norm(U - U_seq) <= 1e-12 * np.linalg.norm(U_seq)


def test_five_level_spatial_coarsening_strategies():
    """Five-level V-cycles with FCF relaxation, m = 4 then 2, and three nested
    meshes 16x64, 8x32, 4x16 (n = 960, 224, 48), with direct spatial
    coarsening (coarse meshes from level 1 on) or delayed spatial coarsening
    (the coarser meshes only on the two coarsest levels, Sec. 2.2, Fig. 5).
    Delayed coarsening converges in about as many iterations as coarsening in
    time only; direct coarsening onto meshes this coarse degrades the
    convergence (the effect the delayed strategy is meant to avoid, Sec. 2.2)
    but, with FCF relaxation, still terminates: the C-relaxation makes one
    more interval of the finest level exact before every restriction, so the
    iterate is exact after N_t / m_0 iterations."""
    fine, mid, coarse = (16, 64), (8, 32), (4, 16)
    out = {}
    for strategy, meshes in (("none", [fine] * 5), ("delayed", [fine, fine, fine, mid, coarse]),
                             ("direct", [fine, mid, coarse, coarse, coarse])):
        cfg = _tiny_cfg(meshes, 256, 4, m_coarse=2)
        H, _ = build(cfg)
        n = H.levels[0].n
        U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
        maxit = cfg.n_steps // cfg.m if strategy == "direct" else 30
        U, hist, conv = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=1e-8 if strategy != "direct" else 0.0,
                                    maxit=maxit)
        out[strategy] = (hist, np.linalg.norm(U - U_seq) / np.linalg.norm(U_seq))
    assert out["delayed"][1] <= 1e-7 and out["none"][1] <= 1e-7
    assert len(out["delayed"][0]) <= len(out["none"][0]) + 2
    assert out["direct"][1] <= 1e-10
    # after as many iterations as delayed coarsening needs, direct coarsening
    # is still far from converged
    k = len(out["delayed"][0]) - 1
    assert out["direct"][0][k] / out["direct"][0][0] > 1e3 * out["delayed"][0][k] / out["delayed"][0][0]
