"""Structure of the P1 operator that the diagonal-window CG kernels rely on,
checked on the oracle's own assembly (eq. 7, Sec. 3.1): with the unknowns of
a polar mesh numbered angle-major (radial fastest, R = n_r - 1 per ray), the
operator M/dt + K is the periodic stencil with offsets {0, +-1, +-R, +-(R+1)}
(mod n), symmetric, and the upper offsets {+1, +R, +R+1} meet every
off-diagonal pair exactly once, so p.Ap = sum_i p_i (a_ii p_i + 2 sum_upper
a_ij p_j)."""

import numpy as np
import pytest

from oracle.fe import MachineFE
from workload import polar_mesh


@pytest.mark.parametrize("nr, nt", [(16, 128), (8, 64), (32, 256)])
def test_angle_major_operator_is_the_periodic_seven_point_stencil(nr, nt):
    fe = MachineFE(polar_mesh(nr, nt))
    dt = 0.02 / 16384
    A = (fe.M / dt + fe.K).tocsr()
    R, n = nr - 1, fe.n
    assert n == R * nt
    a = np.arange(n)
    perm = (a % R) * nt + a // R          # angle-major index -> interior index (radial-major)
    Ap = A[perm][:, perm].tocsr()
    coo = Ap.tocoo()
    nz = coo.data != 0
    offsets = set(((coo.col - coo.row) % n)[nz].tolist())
    assert offsets <= {0, 1, R, R + 1, n - 1, n - R, n - R - 1}
    assert {0, 1, R, R + 1} <= offsets
    asym = abs(Ap - Ap.T).max()
    assert asym <= 1e-12 * abs(Ap).max()
    rng = np.random.default_rng(nr)
    p = rng.standard_normal(n)
    half = Ap.diagonal() * p
    for o in (1, R, R + 1):
        c_o = np.asarray(Ap[a, (a + o) % n]).ravel()
        half = half + 2.0 * c_o * p[(a + o) % n]
    full = p @ (Ap @ p)
    assert abs(p @ half - full) <= 1e-12 * abs(full)
