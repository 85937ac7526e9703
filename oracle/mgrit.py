"""FAS-MGRIT (Algorithm 1) with V-cycle recursion (Sec. 2.1) and spatial coarsening (Sec. 2.2).

Space-time system on level l (N_l steps, points 0..N_l):

    (A_l(u))_0 = u_0,   (A_l(u))_i = u_i - Phi_l(u_{i-1}),   A_l(u) = g.

On the finest level g_0 = u0 and g_i = 0 (the forcing lives inside Phi, as in
the block system of Sec. 2).  Every m-th point is a C-point.

One cycle on level l (`cycle`), following Algorithm 1:
  * F-relaxation, then gamma times C- then F-relaxation (gamma = 1: FCF);
  * C-point residual r_k = g_km - u_km + Phi_l(u_km-1) (k >= 1), r_0 = g_0 - u_0;
    after F-relaxation the F-point residuals are zero;
  * injection of the C-points and spatial restriction:
        u2_k = R_s u_km,
        g2_0 = u2_0 + R_s r_0,   g2_k = u2_k - Phi_{l+1}(u2_{k-1}) + R_s r_k
    (that is g2 = A_{l+1}(u2) + R_s r, the FAS right-hand side);
  * solve A_{l+1}(v) = g2: recursively on intermediate levels (V-cycle), by
    sequential stepping on the coarsest one;
  * e = v - u2, u_km += P_s e_k, then F-relaxation (ideal interpolation).
    On the finest level that F-relaxation is the first one of the next
    iteration (F-relaxation depends on the C-points only, so F F = F).

Iteration (finest level): relax, measure rho = ||r||_2 over every C-point
and DOF, stop when rho <= tol * rho_0 (rho_0 of the first iteration), else
correct.  The returned iterate is the relaxed one of the stopping iteration.
With F- (FCF-) relaxation and no spatial coarsening, the iteration is exact
after N_t/m (N_t/(2m)) iterations (Sec. 2.1).

Cycles (Sec. 2.1, Fig. 4): in a V-cycle the coarse problem of level l is
approximated by one cycle on level l+1; in an F-cycle by an F-cycle on level
l+1 followed by a V-cycle on level l+1 (on the coarsest level, whose solve is
exact, by the one sequential solve).  For four levels an F-cycle visits the
levels 0 1 2 3 2 3 2 1 2 3 2 1 0.

Nested iteration (Sec. 2.1, used for the initial guess in Sec. 4.1): the
time-stepping problem of the coarsest level is solved sequentially, its
points are interpolated to the C-points of the next finer level (P_s in
space), one V-cycle is applied to that level's own problem (g_0 = the
restricted initial value, g_i = 0), and so on up to level 0 -- the F-cycle
without its first descent.  Sec. 4.1 drives this start with the sine
reference signals as the source; the hierarchy passed in carries that source.

Joule losses (Sec. 3.1): P(t_i) = l_z (du/dt)^T M (du/dt) with the sigma-mass
matrix M and the backward difference du/dt = (u_i - u_{i-1}) / dt of the
implicit-Euler grid.  The stop rule of Sec. 5.1 ends the iteration once the
largest relative change of the C-point losses between two successive
iterations is below a threshold (1e-2 in the paper).
"""

import numpy as np


class ExactCoarse:
    """Coarse propagator equal to m fine steps (the 'ideal' coarse operator)."""

    def __init__(self, fine_level, m):
        self.fine, self.m, self.n = fine_level, m, fine_level.n
        self.dt = fine_level.dt * m

    def phi(self, u_prev, i_from):
        u = np.atleast_2d(u_prev).copy()
        base = np.atleast_1d(i_from) * self.m
        for j in range(self.m):
            u = self.fine.phi(u, base + j)
        return u


class Hierarchy:
    """levels[l] has .phi(u [B, n_l], i_from [B]) and .n; R[l], P[l] map l <-> l+1
    (None = same mesh, no spatial transfer).  m is the temporal coarsening
    factor of every level, or a list: m[l] between levels l and l+1 (Sec. 4.2
    coarsens the first level by a large factor and the others by a small one)."""

    def __init__(self, levels, m, R=None, P=None, gamma=1):
        self.levels = levels
        L = len(levels)
        self.ms = list(m) if isinstance(m, (list, tuple)) else [m] * max(L - 1, 1)
        self.m = self.ms[0]
        self.R = R if R is not None else [None] * (L - 1)
        self.P = P if P is not None else [None] * (L - 1)
        self.gamma = gamma
        self.phi_count = [0] * L
        self.cycle = "V"       # or "F"
        self.visits = []       # level of every relaxation / coarsest solve, in order

    def phi(self, l, u, i_from):
        self.phi_count[l] += np.atleast_2d(u).shape[0]
        return self.levels[l].phi(u, i_from)

    @staticmethod
    def _apply(T, x):
        """Apply a spatial transfer to a batch x [B, n] (identity when T is None)."""
        return x.copy() if T is None else (T @ x.T).T


def f_relax(H, l, u, g):
    m, N = H.ms[l], u.shape[0] - 1
    for j in range(1, m):
        idx = np.arange(j, N + 1, m)          # F-points k*m + j
        if idx.size == 0:
            continue
        u[idx] = H.phi(l, u[idx - 1], idx - 1) + g[idx]


def c_relax(H, l, u, g):
    m, N = H.ms[l], u.shape[0] - 1
    idx = np.arange(m, N + 1, m)              # C-points k >= 1
    u[idx] = H.phi(l, u[idx - 1], idx - 1) + g[idx]


def relax(H, l, u, g):
    f_relax(H, l, u, g)
    for _ in range(H.gamma):
        c_relax(H, l, u, g)
        f_relax(H, l, u, g)


def c_residual(H, l, u, g):
    """r [N_T+1, n]: r_0 = g_0 - u_0, r_k = g_km - u_km + Phi(u_km-1)."""
    m, N = H.ms[l], u.shape[0] - 1
    idx = np.arange(m, N + 1, m)
    r = np.zeros((idx.size + 1, u.shape[1]))
    r[0] = g[0] - u[0]
    r[1:] = g[idx] - u[idx] + H.phi(l, u[idx - 1], idx - 1)
    return r


def coarse_correct(H, l, u, g, r, kind="V"):
    m = H.ms[l]
    cidx = np.arange(0, u.shape[0], m)
    u2 = Hierarchy._apply(H.R[l], u[cidx])
    rr = Hierarchy._apply(H.R[l], r)
    g2 = np.empty_like(u2)
    g2[0] = u2[0] + rr[0]
    k = np.arange(1, u2.shape[0])
    g2[1:] = u2[1:] - H.phi(l + 1, u2[:-1], k - 1) + rr[1:]
    v = u2.copy()
    if kind == "F":
        # F-cycle: an F-cycle, then a V-cycle on the coarse problem (one exact
        # solve when the coarse level is the coarsest)
        cycle(H, l + 1, v, g2, "F")
        if l + 1 < len(H.levels) - 1:
            cycle(H, l + 1, v, g2, "V")
    else:
        cycle(H, l + 1, v, g2, "V")
    u[cidx] += Hierarchy._apply(H.P[l], v - u2)


def coarsest_solve(H, l, u, g):
    H.visits.append(l)
    u[0] = g[0]
    for i in range(1, u.shape[0]):
        u[i] = H.phi(l, u[i - 1][None], [i - 1])[0] + g[i]


def cycle(H, l, u, g, kind="V"):
    """One V- or F-cycle on level l (> 0), solving A_l(u) = g approximately, in place."""
    if l == len(H.levels) - 1:
        coarsest_solve(H, l, u, g)
        return
    H.visits.append(l)
    relax(H, l, u, g)
    r = c_residual(H, l, u, g)
    coarse_correct(H, l, u, g, r, kind)
    H.visits.append(l)
    f_relax(H, l, u, g)


def joule_losses(level, u_prev, u, dt, l_z=1.0):
    """P = l_z (du/dt)^T M (du/dt) per row of u [B, n] with du = u - u_prev
    (Sec. 3.1, the loss integral with the sigma-mass matrix of the level)."""
    d = (np.atleast_2d(u) - np.atleast_2d(u_prev)) / dt
    return l_z * np.einsum("bi,bi->b", d, (level.fe.M @ d.T).T)


def c_point_losses(H, u):
    """Joule losses at the C-points k >= 1 of the finest level (u_km against u_km-1)."""
    m, N = H.ms[0], u.shape[0] - 1
    idx = np.arange(m, N + 1, m)
    return joule_losses(H.levels[0], u[idx - 1], u[idx], H.levels[0].dt)


def max_relative_change(p_new, p_old):
    """Largest |p_new - p_old| / |p_new| over the points with p_new != 0 (Sec. 5.1)."""
    p_new, p_old = np.asarray(p_new), np.asarray(p_old)
    nz = p_new != 0.0
    if not nz.any():
        return 0.0 if np.array_equal(p_new, p_old) else np.inf
    return float(np.max(np.abs(p_new[nz] - p_old[nz]) / np.abs(p_new[nz])))


def restrict_down(H, x, l):
    """x on level 0's mesh restricted (R_s) to the mesh of level l."""
    for k in range(l):
        x = Hierarchy._apply(H.R[k], np.atleast_2d(x))[0]
    return x


def nested_iteration(H, u0, n_steps):
    """Initial space-time guess of the finest level by nested iteration:
    coarsest sequential solve, then per finer level interpolation of the
    coarse points to its C-points and one V-cycle on its own problem.  The
    F-points of the result are those of the last cycle's F-relaxation, so
    the returned [(n_steps+1), n0] array is a consistent finest-level
    trajectory of that cycle."""
    L = len(H.levels)
    Ns = [n_steps]
    for l in range(L - 1):
        Ns.append(Ns[-1] // H.ms[l])
    # coarsest problem: g_0 = restricted initial value, g_i = 0
    uc = np.zeros((Ns[-1] + 1, H.levels[-1].n))
    gc = np.zeros_like(uc)
    gc[0] = restrict_down(H, u0, L - 1)
    coarsest_solve(H, L - 1, uc, gc)
    for l in range(L - 2, -1, -1):
        u = np.zeros((Ns[l] + 1, H.levels[l].n))
        g = np.zeros_like(u)
        g[0] = restrict_down(H, u0, l)
        u[::H.ms[l]] = Hierarchy._apply(H.P[l], uc)
        u[0] = g[0]
        cycle(H, l, u, g, "V")
        uc = u
    return uc


def solve(H, u0, n_steps, tol=1e-8, maxit=100, guess=None, callback=None, loss_tol=None,
          losses=None):
    """FAS-MGRIT on the finest level (V- or F-cycles per H.cycle).

    Returns (U [(n_steps+1), n0], history of rho, converged flag).
    `maxit` bounds the number of coarse corrections; the last relaxation is
    always followed by a residual evaluation.  With loss_tol set, the
    iteration stops instead once the C-point Joule losses change by less than
    loss_tol (relative, every C-point) between two successive iterations
    (Sec. 5.1); `losses` (a list) then receives the C-point losses of every
    iteration and the change is measured from the second iteration on.
    """
    n0 = H.levels[0].n
    g = np.zeros((n_steps + 1, n0))
    g[0] = u0
    u = np.zeros((n_steps + 1, n0)) if guess is None else np.array(guess, dtype=np.float64)
    u[0] = u0
    hist = []
    converged = False
    p_prev = None
    for it in range(maxit + 1):
        H.visits.append(0)
        relax(H, 0, u, g)
        r = c_residual(H, 0, u, g)
        rho = float(np.linalg.norm(r))
        hist.append(rho)
        if callback is not None:
            callback(it, u, rho)
        if loss_tol is not None:
            p = c_point_losses(H, u)
            if losses is not None:
                losses.append(p)
            if p_prev is not None and max_relative_change(p, p_prev) < loss_tol:
                converged = True
                break
            p_prev = p
        elif rho == 0.0 or rho <= tol * hist[0]:
            converged = True
            break
        if it == maxit:
            break
        coarse_correct(H, 0, u, g, r, H.cycle)
    return u, hist, converged


def parareal(G, F, u0, n_coarse, n_iter, guess_c=None):
    """Parareal with coarse propagator G and fine propagator F (m fine steps).

    U^{k+1}_{n+1} = G(U^{k+1}_n) + F(U^k_n) - G(U^k_n), U^{k}_0 = u0.
    Returns the list of coarse iterates [U^0, U^1, ..., U^n_iter], each [n_coarse+1, n].
    """
    n = u0.size
    U = np.zeros((n_coarse + 1, n)) if guess_c is None else guess_c.copy()
    U[0] = u0
    out = [U.copy()]
    for _ in range(n_iter):
        ks = np.arange(n_coarse)
        FU = F.phi(U[:-1], ks)
        GU = G.phi(U[:-1], ks)
        Unew = np.zeros_like(U)
        Unew[0] = u0
        for k in range(n_coarse):
            Unew[k + 1] = G.phi(Unew[k][None], [k])[0] + FU[k] - GU[k]
        U = Unew
        out.append(U.copy())
    return out
