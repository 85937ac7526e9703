"""Pins of the oracle's finite elements (Sec. 3.1, eq. 7) against closed forms.

Nothing here re-types the assembly formulas: each check is a property the
exact Galerkin operators must have (patch test, exact integrals of linear
functions, conservation of the source, symmetry/definiteness) or a
convergence rate on a manufactured solution.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workload import polar_mesh, MAT_BAR
from workload.machine import material_arrays, R_IN, R_OUT
from oracle import fe


def test_quadrature_integrates_degree5_exactly():
    # unit right triangle (0,0),(1,0),(0,1): int x^a y^b = a! b! / (a+b+2)!
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2]])
    pts, w = fe.quad_points(xy, tri)
    for a in range(6):
        for b in range(6 - a):
            got = np.sum(w[0] * pts[0, :, 0] ** a * pts[0, :, 1] ** b)
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert got == pytest.approx(exact, rel=1e-13, abs=1e-15)


@pytest.fixture(scope="module")
def mach():
    return fe.MachineFE(polar_mesh(8, 64))


def test_geometry_area_sums_to_polygon(mach):
    m = mach.mesh
    # each cell is a quadrilateral with two chord sides; the annulus polygon area
    n = m.n_theta
    poly = 0.5 * n * math.sin(2 * math.pi / n) * (R_OUT ** 2 - R_IN ** 2)
    assert mach.area.sum() == pytest.approx(poly, rel=1e-13)


def test_stiffness_patch_test(mach):
    """K_full applied to any linear function vanishes (constant nu: exactly zero
    flux balance at nodes not on the boundary); K_full 1 = 0 for any nu."""
    m = mach.mesh
    ones = np.ones(m.n_nodes)
    assert np.abs(mach.K_full @ ones).max() < 1e-9 * np.abs(mach.K_full).max()
    K1 = fe.stiffness(m.xy, m.tri, np.full(m.n_tri, 2.5))
    lin = 0.3 + 1.7 * m.xy[:, 0] - 0.9 * m.xy[:, 1]
    res = K1 @ lin
    interior = m.dirichlet == 0
    assert np.abs(res[interior]).max() < 1e-10 * np.abs(K1).max()


def test_stiffness_energy_of_linear_function(mach):
    """u^T K u = nu * |grad u|^2 * area for u linear (exact)."""
    m = mach.mesh
    K1 = fe.stiffness(m.xy, m.tri, np.full(m.n_tri, 3.0))
    u = 2.0 * m.xy[:, 0] + 5.0 * m.xy[:, 1]
    assert u @ (K1 @ u) == pytest.approx(3.0 * 29.0 * mach.area.sum(), rel=1e-12)


def test_mass_integrates_linear_products(mach):
    """1^T M 1 = sum sigma*area over the bars; 1^T M x = integral of sigma*x."""
    m = mach.mesh
    sig = mach.sigma_cell
    assert np.ones(m.n_nodes) @ (mach.M_full @ np.ones(m.n_nodes)) == pytest.approx(
        np.sum(sig * mach.area), rel=1e-13)
    cx = m.xy[m.tri][:, :, 0].mean(axis=1)
    assert np.ones(m.n_nodes) @ (mach.M_full @ m.xy[:, 0]) == pytest.approx(
        np.sum(sig * mach.area * cx), rel=1e-12, abs=1e-9)


def test_operators_symmetric_definite(mach):
    K, M = mach.K.toarray(), mach.M.toarray()
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(K).min() > 0                 # SPD after the Dirichlet elimination
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > -1e-9 * ev.max()                      # PSD
    bar_nodes = np.unique(mach.mesh.tri[mach.mesh.cell_mat == MAT_BAR])
    free = set(mach.free.tolist())
    n_bar_free = sum(1 for v in bar_nodes if v in free)
    assert np.sum(ev > 1e-9 * ev.max()) == n_bar_free     # rank = bar node count
    assert n_bar_free > 0


def test_source_conservation(mach):
    """1^T F_p = sum over phase-p coil cells of sign * area (the total current)."""
    m = mach.mesh
    for p in range(3):
        sel = m.cell_phase == p
        assert sel.any()
        assert mach.F_full[p].sum() == pytest.approx(np.sum(m.cell_sign[sel] * mach.area[sel]), rel=1e-13)
        # balanced winding: each phase has as many + as - coil area
        assert abs(mach.F_full[p].sum()) < 1e-12


def _manufactured(n_r, n_theta, nu, sigma=0.0, gfun=None, dt=None, n_steps=0):
    """Solve -div(nu grad A) (+ sigma dA/dt) = J for A = S(r) cos(2 theta) g(t)."""
    L = R_OUT - R_IN
    k = math.pi / L

    def S(r):
        return np.sin(k * (r - R_IN))

    def lap(x, y):
        r = np.hypot(x, y)
        th = np.arctan2(y, x)
        s, ds, d2s = S(r), k * np.cos(k * (r - R_IN)), -k * k * S(r)
        return (d2s + ds / r - 4.0 * s / r ** 2) * np.cos(2 * th)

    def exact(x, y):
        return S(np.hypot(x, y)) * np.cos(2 * np.arctan2(y, x))

    mesh = polar_mesh(n_r, n_theta)
    K = fe.stiffness(mesh.xy, mesh.tri, np.full(mesh.n_tri, nu))
    free = mesh.interior_nodes()
    Kf = K[free][:, free].tocsc()
    if sigma == 0.0:
        f = fe.load_function(mesh.xy, mesh.tri, lambda x, y: -nu * lap(x, y))
        u = np.zeros(mesh.n_nodes)
        u[free] = spla.spsolve(Kf, f[free])
        gT = 1.0
    else:
        M = fe.mass(mesh.xy, mesh.tri, np.full(mesh.n_tri, sigma))[free][:, free].tocsc()
        lu = spla.splu((M / dt + Kf).tocsc())
        fs = fe.load_function(mesh.xy, mesh.tri, exact)[free]          # int S*cos*phi
        fl = fe.load_function(mesh.xy, mesh.tri, lambda x, y: -lap(x, y))[free]
        uf = np.zeros(free.size)   # g(0) = 0
        for i in range(1, n_steps + 1):
            t = i * dt
            g, dg = gfun(t)
            f = sigma * dg * fs + nu * g * fl
            uf = lu.solve(M @ uf / dt + f)
        u = np.zeros(mesh.n_nodes)
        u[free] = uf
        gT = gfun(n_steps * dt)[0]
    # L2 error by 7-point quadrature of (A_h - A)^2
    pts, w = fe.quad_points(mesh.xy, mesh.tri)
    uh = np.einsum("qa,ta->tq", fe.QUAD7_BARY, u[mesh.tri])
    err = uh - gT * exact(pts[..., 0], pts[..., 1])
    return math.sqrt(np.sum(w * err ** 2))


def test_manufactured_steady_h2_rate():
    errs = [_manufactured(nr, nt, nu=795.0) for nr, nt in [(8, 64), (16, 128), (32, 256), (64, 512)]]
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert rates[-1] == pytest.approx(4.0, abs=0.05), rates
    assert rates[-2] == pytest.approx(4.0, abs=0.1), rates


def test_manufactured_transient_rate():
    """sigma dA/dt - nu lap A = J with A = S cos(2 theta) sin(2 pi 50 t);
    implicit Euler with dt ~ h^2 keeps the O(h^2) L2 rate."""
    w = 2 * math.pi * 50.0
    gfun = lambda t: (math.sin(w * t), w * math.cos(w * t))
    errs = []
    for level, (nr, nt) in enumerate([(8, 64), (16, 128), (32, 256)]):
        n_steps = 8 * 4 ** level
        dt = 0.005 / n_steps
        errs.append(_manufactured(nr, nt, nu=795.0, sigma=1e5, gfun=gfun, dt=dt, n_steps=n_steps))
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert rates[-1] == pytest.approx(4.0, abs=0.1), rates
