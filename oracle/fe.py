"""P1 finite elements for the 2D eddy-current problem (Sec. 3.1).

The field equation of the rotor/stator model reduces, without circuit
coupling and with a fixed rotor, to

    sigma dA/dt - div(nu grad A) = J_s(t),   A = 0 on both radii,

whose Galerkin discretisation with piecewise-linear triangles is the
semi-discrete system M u' + K(u) u = f(t) of eq. 7:

    K_ab = sum_e nu_e * area_e * grad(phi_a) . grad(phi_b)
    M_ab = sum_e sigma_e * area_e / 12 * (1 + delta_ab)      (consistent mass)
    f_a  = sum_e integral_e J phi_a  (= J_e area_e / 3 for a cellwise-constant J)

Dirichlet nodes are removed (their value is 0, so no lifting term appears).
Saturating iron uses nu(B^2) = k1 exp(k2 B^2) + k3 with B^2 = |grad A|^2 on
each element (Brauer law in SI units).
"""

import numpy as np
import scipy.sparse as sp

from workload.machine import material_arrays


def element_geometry(xy, tri):
    """Areas [T] and basis-function gradients [T, 3, 2] of every triangle."""
    p = xy[tri]                      # [T, 3, 2]
    x, y = p[..., 0], p[..., 1]
    # b_a = y_{a+1} - y_{a+2}, c_a = x_{a+2} - x_{a+1} (indices mod 3)
    b = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], axis=1)
    c = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], axis=1)
    two_area = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    if np.any(two_area <= 0):
        raise ValueError("triangles must be counter-clockwise and non-degenerate")
    area = 0.5 * two_area
    grad = np.stack([b, c], axis=2) / two_area[:, None, None]
    return area, grad


def _scatter(tri, vals, n_nodes):
    """Sum element matrices vals[T, 3, 3] into a sparse N x N matrix."""
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    return sp.csr_matrix((vals.ravel(), (rows, cols)), shape=(n_nodes, n_nodes))


def stiffness(xy, tri, nu_cell):
    area, grad = element_geometry(xy, tri)
    ke = np.einsum("t,tad,tbd->tab", nu_cell * area, grad, grad)
    return _scatter(tri, ke, xy.shape[0])


def mass(xy, tri, sigma_cell):
    area, _ = element_geometry(xy, tri)
    local = (np.ones((3, 3)) + np.eye(3)) / 12.0
    me = (sigma_cell * area)[:, None, None] * local[None]
    return _scatter(tri, me, xy.shape[0])


def load_cellwise(xy, tri, j_cell):
    """f_a = sum_e J_e area_e / 3 over the elements touching node a."""
    area, _ = element_geometry(xy, tri)
    f = np.zeros(xy.shape[0])
    np.add.at(f, tri.ravel(), np.repeat(j_cell * area / 3.0, 3))
    return f


# Degree-5, 7-point symmetric quadrature rule on the triangle (Dunavant 1985),
# barycentric coordinates and weights (weights sum to 1, multiply by area).
_A1, _B1, _W1 = 0.059715871789770, 0.470142064105115, 0.132394152788506
_A2, _B2, _W2 = 0.797426985353087, 0.101286507323456, 0.125939180544827
QUAD7_BARY = np.array([
    [1 / 3, 1 / 3, 1 / 3],
    [_A1, _B1, _B1], [_B1, _A1, _B1], [_B1, _B1, _A1],
    [_A2, _B2, _B2], [_B2, _A2, _B2], [_B2, _B2, _A2],
])
QUAD7_W = np.array([0.225, _W1, _W1, _W1, _W2, _W2, _W2])


def quad_points(xy, tri):
    """Physical quadrature points [T, 7, 2] and weights*area [T, 7]."""
    area, _ = element_geometry(xy, tri)
    pts = np.einsum("qa,tad->tqd", QUAD7_BARY, xy[tri])
    return pts, area[:, None] * QUAD7_W[None, :]


def load_function(xy, tri, jfun):
    """f_a = integral of J(x, y) * phi_a, by 7-point quadrature per element."""
    pts, w = quad_points(xy, tri)
    jv = jfun(pts[..., 0], pts[..., 1])           # [T, 7]
    fe = np.einsum("tq,qa->ta", jv * w, QUAD7_BARY)
    f = np.zeros(xy.shape[0])
    np.add.at(f, tri.ravel(), fe.ravel())
    return f


class MachineFE:
    """Interior-node operators of the synthetic machine on one mesh."""

    def __init__(self, mesh):
        self.mesh = mesh
        nu_mat, sig_mat, iron_mat = material_arrays()
        self.nu_cell = nu_mat[mesh.cell_mat]
        self.sigma_cell = sig_mat[mesh.cell_mat]
        self.iron_cell = iron_mat[mesh.cell_mat].astype(bool)
        self.area, self.grad = element_geometry(mesh.xy, mesh.tri)
        self.free = mesh.interior_nodes()
        self.n = self.free.size
        K = stiffness(mesh.xy, mesh.tri, self.nu_cell)
        M = mass(mesh.xy, mesh.tri, self.sigma_cell)
        self.K_full, self.M_full = K, M
        self.K = K[self.free][:, self.free].tocsr()
        self.M = M[self.free][:, self.free].tocsr()
        # one load vector per phase, for unit current density times the winding sign
        F = []
        for p in range(3):
            jc = np.where(mesh.cell_phase == p, mesh.cell_sign, 0).astype(np.float64)
            F.append(load_cellwise(mesh.xy, mesh.tri, jc))
        self.F_full = np.stack(F)            # [3, N]
        self.F = self.F_full[:, self.free]   # [3, n]

    def to_full(self, u):
        """Interior vector(s) [..., n] -> nodal vector(s) [..., N] with zeros on the boundary."""
        out = np.zeros(u.shape[:-1] + (self.mesh.n_nodes,))
        out[..., self.free] = u
        return out

    # --- saturating iron (nonlinear model) ---------------------------------
    def b_squared(self, u):
        """|grad A|^2 per element for an interior vector u."""
        a = self.to_full(u)[self.mesh.tri]            # [T, 3]
        g = np.einsum("ta,tad->td", a, self.grad)     # [T, 2]
        return np.sum(g * g, axis=1)

    def nu_nonlinear(self, b2, bh):
        """nu_e and d nu / d(B^2) per element (linear nu outside the iron)."""
        nu = self.nu_cell.copy()
        dnu = np.zeros_like(nu)
        e = np.exp(bh.k2 * b2[self.iron_cell])
        nu[self.iron_cell] = bh.k1 * e + bh.k3
        dnu[self.iron_cell] = bh.k1 * bh.k2 * e
        return nu, dnu

    def stiffness_nonlinear(self, u, bh):
        """K(u): stiffness with nu evaluated at the element fields of u."""
        nu, _ = self.nu_nonlinear(self.b_squared(u), bh)
        K = stiffness(self.mesh.xy, self.mesh.tri, nu)
        return K[self.free][:, self.free].tocsr()

    def jacobian_nonlinear(self, u, bh):
        """d(K(u) u)/du = sum_e [nu_e G_e + 2 nu'_e / area_e (G_e u_e)(G_e u_e)^T],

        with G_e = area_e grad(phi) grad(phi)^T, because
        B_e^2 = u_e^T G_e u_e / area_e.
        """
        nu, dnu = self.nu_nonlinear(self.b_squared(u), bh)
        G = np.einsum("t,tad,tbd->tab", self.area, self.grad, self.grad)
        ue = self.to_full(u)[self.mesh.tri]
        Gu = np.einsum("tab,tb->ta", G, ue)
        je = nu[:, None, None] * G + (2.0 * dnu / self.area)[:, None, None] * Gu[:, :, None] * Gu[:, None, :]
        J = _scatter(self.mesh.tri, je, self.mesh.n_nodes)
        return J[self.free][:, self.free].tocsr()
