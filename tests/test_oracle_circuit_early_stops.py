"""Early-stopped linear solves in the field-circuit coupled step (Sec. 3.1)
inside MGRIT (Algorithm 1), emulated on the CPU with the oracle's matrices.

The GPU path solves each coupled step as A y = (M/dt) a, eliminates the k
circuit unknowns w and returns a' = y + Z w (Z = A^-1 B^T).  When the solve for
y stops early, two choices decide whether MGRIT still converges:
- the start of the solve: from a guess of a' the start residual holds the
  circuits' field B^T w, so a stop at eta times it leaves an error that does
  not shrink with the iterations; from the guess less Z times the circuit
  unknowns of the previous step from the same time point it does shrink;
- the circuit rows after an inexact solve: with A symmetric, B A^-1 r = Z^T r
  for the solve's residual r, so the exact B (y* - a) is B (y - a) + Z^T r;
  without that term the elimination multiplies the solve's error.
This test runs the oracle's MGRIT with level 0 stepped by such inexact solves
(Jacobi-PCG) and checks all three outcomes.  It pins the reading behind the
coupled solves' start and the residual term of the elimination; it does not
call the GPU path."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workload import config, Circuit
from workload.configs import LevelSpec
from oracle.problem import build
from oracle import mgrit, stepping

N_STEPS = 256
ETA, ETA_R = 3e-3, 1e-4


class InexactCoupledLevel:
    """phi(u_prev, i_from) of a coupled level with an early-stopped Jacobi-PCG
    solve for y and the elimination of the circuit unknowns; keeps, per time
    point, the last output and circuit unknowns as the next start."""

    def __init__(self, lev, eta, stored_start, residual_term, tol):
        self.lev, self.n = lev, lev.n
        self.eta, self.eta_now = eta, eta
        self.stored_start, self.residual_term, self.tol = stored_start, residual_term, tol
        c = lev.circuit
        self.A = lev.A
        self.dinv = 1.0 / lev.A.diagonal()
        self.B = np.vstack([lev.X, lev.Yp / c.l_z])
        k = self.B.shape[0]
        self.Z = spla.splu(lev.A.tocsc()).solve(np.ascontiguousarray(self.B.T))
        self.f = c.l_z / lev.dt
        self.E = np.diag([1.0] * 3 + [-1.0] * lev.nb)
        D = np.zeros((k, k))
        D[:3, :3] = c.r_phase * np.eye(3)
        if lev.nb:
            D[3:, 3:] = lev.C
        self.S = self.f * self.E @ self.B @ self.Z + D
        self.k = k
        self.prev_a, self.prev_w = {}, {}
        self.cg_iterations = 0

    def _pcg(self, b, X):
        R = b - self.A @ X
        bn = np.linalg.norm(b, axis=0)
        r0 = np.linalg.norm(R, axis=0)
        thr = np.maximum(self.tol * np.where(bn > 0, bn, r0), self.eta_now * r0)
        Zp = self.dinv[:, None] * R
        P = Zp.copy()
        rz = np.sum(R * Zp, axis=0)
        act = r0 > thr
        while act.any():
            self.cg_iterations += int(act.sum())
            AP = self.A @ P
            pap = np.sum(P * AP, axis=0)
            al = np.where(act, rz / np.where(pap != 0, pap, 1.0), 0.0)
            X += al * P
            R -= al * AP
            Zp = self.dinv[:, None] * R
            rz_new = np.sum(R * Zp, axis=0)
            be = np.where(act, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
            rz = rz_new
            P = np.where(act, Zp + be * P, P)
            act &= np.linalg.norm(R, axis=0) > thr
        return X

    def phi(self, u_prev, i_from):
        u_prev, i_from = np.atleast_2d(u_prev), np.atleast_1d(i_from)
        lev = self.lev
        b = lev.Mdt @ u_prev.T
        X = np.empty((self.n, u_prev.shape[0]))
        for c, i in enumerate(i_from):
            X[:, c] = self.prev_a.get(int(i), u_prev[c])
            if self.stored_start and int(i) in self.prev_w:
                X[:, c] -= self.Z @ self.prev_w[int(i)]
        Y = self._pcg(b, X)
        t = (i_from.astype(np.float64) + 1.0) * lev.dt
        rhs = np.zeros((self.k, u_prev.shape[0]))
        rhs[:3] = lev.voltages(t).T
        d = self.B @ (Y - u_prev.T)
        if self.residual_term:
            d += self.Z.T @ (b - self.A @ Y)
        W = np.linalg.solve(self.S, rhs - self.f * self.E @ d)
        out = Y + self.Z @ W
        for c, i in enumerate(i_from):
            self.prev_a[int(i)] = out[:, c].copy()
            self.prev_w[int(i)] = W[:, c].copy()
        return out.T


@pytest.fixture(scope="module")
def problem():
    cfg = config("cfg1", circuit=Circuit(), n_steps=N_STEPS, t_final=N_STEPS * 0.01 / 512)
    cfg.meshes = [LevelSpec(16, 128), LevelSpec(8, 64)]
    H, _ = build(cfg)
    U_seq = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), N_STEPS)
    return cfg, U_seq


def _solve(cfg, eta, stored_start, residual_term, tol, maxit, monkeypatch):
    H, _ = build(cfg)
    n = H.levels[0].n
    lev = InexactCoupledLevel(H.levels[0], eta, stored_start, residual_term, tol)
    H.levels[0] = lev
    orig = mgrit.c_residual

    def c_residual(H_, l, u, g):
        # the C-point residual solves stop at ETA_R of their start residual
        keep = lev.eta_now
        lev.eta_now = ETA_R if (l == 0 and eta > 0) else keep
        try:
            return orig(H_, l, u, g)
        finally:
            lev.eta_now = keep

    monkeypatch.setattr(mgrit, "c_residual", c_residual)
    with np.errstate(over="ignore", invalid="ignore"):
        U, hist, conv = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=cfg.mgrit_tol, maxit=maxit)
    return U, hist, conv, lev.cg_iterations


def test_early_stops_from_the_stored_start_converge(problem, monkeypatch):
    cfg, U_seq = problem
    _, hist_s, conv_s, cg_strict = _solve(cfg, 0.0, False, True, 1e-12, 30, monkeypatch)
    U, hist, conv, cg = _solve(cfg, ETA, True, True, 1e-14, 30, monkeypatch)
    assert conv_s and conv
    assert len(hist) <= len(hist_s) + 3, (len(hist), len(hist_s))
    assert cg < 0.4 * cg_strict, (cg, cg_strict)
    err = np.linalg.norm(U - U_seq, axis=1)[1:] / np.linalg.norm(U_seq, axis=1)[1:]
    assert err.max() <= 1e-7, err.max()


def test_early_stops_from_a_guess_of_a_stall(problem, monkeypatch):
    cfg, _ = problem
    _, hist, conv, _ = _solve(cfg, ETA, False, True, 1e-14, 12, monkeypatch)
    assert not conv
    # the iteration levels off on the order of eta (of rho_0)
    tail = np.array(hist[-4:]) / hist[0]
    assert tail.min() > 1e-3 and tail.max() < 3e-2, tail


def test_early_stops_without_the_residual_term_diverge(problem, monkeypatch):
    cfg, _ = problem
    _, hist, conv, _ = _solve(cfg, ETA, True, False, 1e-14, 6, monkeypatch)
    assert not conv
    assert not np.isfinite(hist[-1]) or hist[-1] > 1e6 * hist[0], hist
