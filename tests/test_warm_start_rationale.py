"""Why the level-0 F-relaxation solves may start from u_j^old + (u_{j-1} -
u_{j-1}^old) (warm_start = 2): at the machine's small time steps the
propagator Phi acts almost as the identity on slowly varying changes, so
u_j^old = Phi(u_{j-1}^old) plus the input change is much closer to
Phi(u_{j-1}) than u_j^old alone.  Checked on the oracle's exact-solve MGRIT
(Algorithm 1) for the F-points j >= 2 of every relaxation after the first."""

import numpy as np

from oracle import mgrit
from oracle.problem import build
from workload import config


def test_input_change_start_is_much_closer_than_the_previous_iterate():
    cfg = config("cfg1", n_steps=512, t_final=0.02 * 512 / 16384)   # 16x128, headline dt
    H, _ = build(cfg)
    L0 = H.levels[0]
    A = L0.A.tocsr()
    s = 1.0 / np.sqrt(A.diagonal())
    N, m = cfg.n_steps, cfg.m
    inp = {}
    ratios = []
    orig = mgrit.f_relax

    def f_relax(Hh, l, u, g):
        if l != 0:
            return orig(Hh, l, u, g)
        for j in range(1, m):
            idx = np.arange(j, N + 1, m)
            b = L0.rhs(u[idx - 1], idx - 1)
            if j >= 2 and all(int(i) in inp for i in idx):
                prev = np.stack([inp[int(i)] for i in idx])
                r_old = np.linalg.norm(s * (b - (A @ u[idx].T).T), axis=1)
                r_new = np.linalg.norm(s * (b - (A @ (u[idx] + u[idx - 1] - prev).T).T), axis=1)
                ok = r_old > 0
                ratios.append(np.median(r_new[ok] / r_old[ok]))
            for i in idx:
                inp[int(i)] = u[i - 1].copy()
            u[idx] = L0.lu.solve(b.T).T + g[idx]

    mgrit.f_relax = f_relax
    try:
        mgrit.solve(H, np.zeros(L0.n), N, tol=1e-8, maxit=4)
    finally:
        mgrit.f_relax = orig
    assert len(ratios) > 0
    assert np.median(ratios) < 0.1, ratios
