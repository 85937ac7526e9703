"""Implicit Euler propagator Phi and sequential time stepping (Sec. 2, eq. 2; Sec. 3.1, eq. 8).

One step of backward Euler for M u' + K(u) u = f(t) from t_{i-1} to t_i:

    (M/dt + K(u_i)) u_i = f(t_i) + (M/dt) u_{i-1}.

The printed eq. 8 has 1/Delta T on the mass term of the right-hand side;
it is read as the level's own step dt on both sides (otherwise the scheme is
not backward Euler).  The source is sampled at the new time t_i = i*dt,
computed as a product, never by accumulation.

Linear model: one sparse LU factorisation per level, reused by every step.
Nonlinear model: damped Newton (Sec. 5.1: the nonlinear solves use Newton's
method with damping) with the exact Jacobian, initial guess u_{i-1}, one
direct solve per Newton step.  The paper does not say how it damps; the step
length is chosen by the Armijo rule on the residual norm (Kelley, Iterative
Methods for Linear and Nonlinear Equations, SIAM 1995, Sec. 8.1): the first
lambda in 1, 1/2, ..., 2**-halvings with
||R(u - lambda d)|| < (1 - 1e-4 lambda) ||R(u)||, else the last one tried
(a trial whose residual is not finite is rejected).  Stop when
||R(u^k)||_2 <= tol * ||R(u^0)||_2, at most `maxit` Newton steps.
"""

import numpy as np
import scipy.sparse.linalg as spla

from . import pwm
from .fe import MachineFE


class NewtonFailure(RuntimeError):
    pass


class Level:
    """The propagator of one MGRIT level: a mesh, a step size and the source."""

    def __init__(self, mesh, dt, source, bh=None, fe=None, newton_tol=1e-10,
                 newton_maxit=8, newton_halvings=6):
        self.fe = fe if fe is not None else MachineFE(mesh)
        self.n = self.fe.n
        self.dt = dt
        self.source = source
        self.bh = bh
        self.nonlinear = bool(bh is not None and bh.nonlinear)
        self.newton_tol = newton_tol
        self.newton_maxit = newton_maxit
        self.newton_halvings = newton_halvings
        self.Mdt = (self.fe.M / dt).tocsr()
        self.newton_iters = []
        self.newton_lambdas = []
        if not self.nonlinear:
            self.A = (self.Mdt + self.fe.K).tocsc()
            self.lu = spla.splu(self.A)

    def forcing(self, t):
        """f(t) for a vector of times t [B]: [B, n]."""
        b = pwm.phase_signals(t, self.source)            # [3, B]
        s = self.source.J0 * self.source.amplitude * pwm.ramp(t, self.source)
        return s[:, None] * (b.T @ self.fe.F)

    def rhs(self, u_prev, i_from):
        """(M/dt) u_prev + f(t_{i_from+1}) for each column of the batch."""
        t = (np.asarray(i_from, dtype=np.float64) + 1.0) * self.dt
        return (self.Mdt @ u_prev.T).T + self.forcing(t)

    def residual(self, u, u_prev, f):
        """R(u) = (M/dt)(u - u_prev) + K(u) u - f for one column."""
        return self.Mdt @ (u - u_prev) + self.fe.stiffness_nonlinear(u, self.bh) @ u - f

    def newton(self, u_prev, f):
        u = u_prev.copy()
        r = self.residual(u, u_prev, f)
        r0 = np.linalg.norm(r)
        if r0 == 0.0:
            self.newton_iters.append(0)
            return u
        rn = r0
        for k in range(1, self.newton_maxit + 1):
            J = (self.Mdt + self.fe.jacobian_nonlinear(u, self.bh)).tocsc()
            d = spla.spsolve(J, r)
            lam = 1.0
            for h in range(self.newton_halvings + 1):
                lam = 0.5 ** h
                with np.errstate(over="ignore", invalid="ignore"):
                    u_try = u - lam * d
                    r_try = self.residual(u_try, u_prev, f)
                    rn_try = np.linalg.norm(r_try)
                if np.isfinite(rn_try) and rn_try < (1.0 - 1e-4 * lam) * rn:
                    break
            if not np.isfinite(rn_try):
                raise NewtonFailure("non-finite residual at the shortest damped step")
            u, r, rn = u_try, r_try, rn_try
            self.newton_lambdas.append(lam)
            if rn <= self.newton_tol * r0:
                self.newton_iters.append(k)
                return u
        raise NewtonFailure(f"Newton did not reach {self.newton_tol} in {self.newton_maxit} iterations")

    def phi(self, u_prev, i_from):
        """Phi applied to a batch: u_prev [B, n], i_from [B] -> u [B, n] at t_{i_from+1}."""
        u_prev = np.atleast_2d(u_prev)
        i_from = np.atleast_1d(i_from)
        b = self.rhs(u_prev, i_from)
        if not self.nonlinear:
            return self.lu.solve(np.ascontiguousarray(b.T)).T
        t = (i_from.astype(np.float64) + 1.0) * self.dt
        f = self.forcing(t)
        return np.stack([self.newton(u_prev[k], f[k]) for k in range(u_prev.shape[0])])


def sequential(level, u0, n_steps):
    """Forward block solve of the space-time system: U [(n_steps+1), n]."""
    U = np.zeros((n_steps + 1, level.n))
    U[0] = u0
    for i in range(1, n_steps + 1):
        U[i] = level.phi(U[i - 1][None], [i - 1])[0]
    return U
