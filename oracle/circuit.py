"""Field-circuit coupled implicit Euler step (Sec. 3.1, the stator and rotor
circuit equations of the eddy-current system; Sec. 3.2 voltage source; eq. 8).

Test infrastructure: the CPU oracle.  Only tests/, the smoke check and the
benchmark's CPU leg use this module; the library never does.

Unknowns of one step from t_{i-1} to t_i: the vector potential a (n interior
nodes), the stator phase currents i1 (3) and the rotor bar voltages v2 (n_b).

Stator, stranded conductors.  The winding function of phase s is
turns_density * sign on the cells of phase s, so its load vector is
X_s = turns_density * F_s (F_s: the unit current-density load vector) and
its flux linkage l_z X_s^T a.  The coil equation, with the phase resistance
R and the source voltage v_s(t) = v0 * amplitude * ramp(t) * b_s(t):
    l_z X_s^T (a_i - a_{i-1}) / dt + R i1_s = v_s(t_i).
Rotor, solid conductors.  The voltage distribution function of bar k is
1 / l_z on the bar, so bar k adds sigma v_k / l_z as a current density:
its field coupling is Y_k = Y'_k / l_z with Y'_k = integral of sigma phi over
the bar, and its current is
    i2_k = G_k v_k - Y'_k^T (a_i - a_{i-1}) / dt,   G_k = sigma area_k / l_z.
End rings (the inductive-circuit relation, read as a resistive ladder; no
ring inductance, so every circuit unknown is algebraic): two rings with
resistance ring_r between neighbouring bars, symmetric about the bars, give
i2 = -(1 / (2 ring_r)) L v2, L the periodic path Laplacian over the bars.
Together:  C v2 = Y'^T (a_i - a_{i-1}) / dt  with  C = diag(G) + L / (2 ring_r).

Field rows (the semi-discrete eq. 7 with the circuit terms):
    (M/dt + K) a_i - X^T i1 - Y^T v2 = (M/dt) a_{i-1}.

The bordered system of a, i1, v2 is assembled as one sparse matrix and
factorised once per level (SuperLU); every step is one solve.  MGRIT's state
is a alone: the circuit unknowns follow from a_i and a_{i-1}.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import pwm
from .fe import MachineFE, load_cellwise


def ring_laplacian(nb):
    """Periodic path Laplacian over nb bars: 2 on the diagonal, -1 between
    neighbours k, k+1 (mod nb)."""
    L = 2.0 * np.eye(nb)
    for k in range(nb):
        L[k, (k + 1) % nb] -= 1.0
        L[(k + 1) % nb, k] -= 1.0
    return L


def cage_matrix(G, ring_r):
    """C = diag(G) + L / (2 ring_r): bar voltages from the bars' EMF terms."""
    G = np.asarray(G, dtype=np.float64)
    return np.diag(G) + ring_laplacian(G.size) / (2.0 * ring_r)


class CircuitLevel:
    """The propagator of one MGRIT level of the field-circuit coupled model
    (linear materials).  Same interface as stepping.Level: phi(u_prev, i_from)."""

    nonlinear = False

    def __init__(self, mesh, dt, source, circuit, fe=None):
        self.fe = fe if fe is not None else MachineFE(mesh)
        self.n = self.fe.n
        self.dt = dt
        self.source = source
        self.circuit = c = circuit
        self.Mdt = (self.fe.M / dt).tocsr()
        self.A = (self.Mdt + self.fe.K).tocsr()
        self.X = c.turns_density * self.fe.F                      # [3, n]
        nb = c.n_bars if c.rotor else 0
        self.nb = nb
        Yp, G = [], []
        for k in range(nb):
            on = (mesh.cell_bar == k).astype(np.float64)
            Yp.append(load_cellwise(mesh.xy, mesh.tri, self.fe.sigma_cell * on)[self.fe.free])
            G.append(float(np.sum(self.fe.sigma_cell * on * self.fe.area)) / c.l_z)
        self.Yp = np.array(Yp).reshape(nb, self.n)                 # [nb, n]
        self.G = np.array(G)
        self.C = cage_matrix(self.G, c.ring_r) if nb else np.zeros((0, 0))
        k = 3 + nb
        B = np.vstack([self.X, self.Yp / c.l_z])                   # field couplings [k, n]
        top = sp.hstack([self.A, sp.csr_matrix(-B.T)])
        stator = sp.hstack([sp.csr_matrix(c.l_z / dt * self.X),
                            sp.csr_matrix(np.hstack([c.r_phase * np.eye(3), np.zeros((3, nb))]))])
        rows = [top, stator]
        if nb:
            rows.append(sp.hstack([sp.csr_matrix(-self.Yp / dt),
                                   sp.csr_matrix(np.hstack([np.zeros((nb, 3)), self.C]))]))
        self.big = sp.vstack(rows).tocsc()
        assert self.big.shape == (self.n + k, self.n + k)
        self.lu = spla.splu(self.big)

    def voltages(self, t):
        """Phase voltages v_s(t) for a vector of times: [B, 3]."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        b = pwm.phase_signals(t, self.source)                       # [3, B]
        s = self.circuit.v0 * self.source.amplitude * pwm.ramp(t, self.source)
        return (s[None, :] * b).T

    def step(self, u_prev, i_from):
        """One coupled step for a batch: (a [B, n], i1 [B, 3], v2 [B, nb])."""
        u_prev = np.atleast_2d(u_prev)
        i_from = np.atleast_1d(i_from)
        c = self.circuit
        t = (i_from.astype(np.float64) + 1.0) * self.dt
        rhs = [(self.Mdt @ u_prev.T), self.voltages(t).T + c.l_z / self.dt * (self.X @ u_prev.T)]
        if self.nb:
            rhs.append(-(self.Yp @ u_prev.T) / self.dt)
        sol = self.lu.solve(np.ascontiguousarray(np.vstack(rhs)))
        n = self.n
        return sol[:n].T, sol[n:n + 3].T, sol[n + 3:].T

    def phi(self, u_prev, i_from):
        """Phi applied to a batch: u_prev [B, n], i_from [B] -> u [B, n] at t_{i_from+1}."""
        return self.step(u_prev, i_from)[0]

    def circuit_values(self, u_prev, u, i_from):
        """Stator currents, bar voltages and bar currents of the steps
        u_prev -> u (rows of [B, n]), from the circuit equations alone:
        (i1 [B, 3], v2 [B, nb], i2 [B, nb])."""
        c = self.circuit
        u_prev, u = np.atleast_2d(u_prev), np.atleast_2d(u)
        t = (np.atleast_1d(i_from).astype(np.float64) + 1.0) * self.dt
        du = (u - u_prev) / self.dt
        i1 = (self.voltages(t) - c.l_z * du @ self.X.T) / c.r_phase
        if not self.nb:
            z = np.zeros((u.shape[0], 0))
            return i1, z, z
        v2 = np.linalg.solve(self.C, (du @ self.Yp.T).T).T
        i2 = -(v2 @ ring_laplacian(self.nb).T) / (2.0 * c.ring_r)
        return i1, v2, i2
