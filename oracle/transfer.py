"""Spatial grid transfers between nested polar meshes (Sec. 2.2 and Sec. 3.4).

The paper uses standard finite-element (nodal) interpolation as the
prolongation P_s.  On the curved annulus the fine mid-edge nodes do not lie
on the coarse chords, so P_s is read as P1 interpolation in the logical
(i, j) coordinates of the nested structured mesh: fine node (I, J) sits at
logical point (I/2, J/2) of the coarse mesh and takes the values of the
coarse triangle containing it, weighted by its barycentric coordinates.

The restriction is the row-normalised transpose R_s = D^{-1} P_s^T
(D = row sums of P_s^T), applied to both the state and the residual of the
FAS coarse problem; the MGRIT residual is state-valued (u - Phi(u)), so an
unnormalised P_s^T would scale it by about 4.  Plain P_s^T and injection are
kept as alternatives.  The FAS fixed point does not depend on this choice.
"""

import numpy as np
import scipy.sparse as sp


def _interior_index(mesh):
    idx = -np.ones(mesh.n_nodes, dtype=np.int64)
    free = mesh.interior_nodes()
    idx[free] = np.arange(free.size)
    return idx


def check_nested(fine, coarse):
    if fine.n_r != 2 * coarse.n_r or fine.n_theta != 2 * coarse.n_theta:
        raise ValueError("meshes are not nested (need n_r, n_theta doubled)")
    ci, cj = np.meshgrid(np.arange(coarse.n_r + 1), np.arange(coarse.n_theta), indexing="ij")
    fine_ids = (2 * ci) * fine.n_theta + 2 * cj
    if not np.allclose(fine.xy[fine_ids.ravel()], coarse.xy, rtol=0, atol=1e-12):
        raise ValueError("coarse nodes do not coincide with even fine nodes")


def prolongation(fine, coarse):
    """P_s: interior coarse values -> interior fine values (sparse n_f x n_c)."""
    check_nested(fine, coarse)
    fidx = _interior_index(fine)
    cidx = _interior_index(coarse)
    ntc = coarse.n_theta
    rows, cols, vals = [], [], []
    for node in fine.interior_nodes():
        I, J = divmod(int(node), fine.n_theta)
        # logical position in the coarse mesh
        s_abs, q_abs = I / 2.0, J / 2.0
        i0 = min(int(np.floor(s_abs)), coarse.n_r - 1)
        j0 = int(np.floor(q_abs))
        s, q = s_abs - i0, q_abs - j0
        if s >= q:   # lower triangle [(i,j), (i+1,j), (i+1,j+1)]
            verts = [(i0, j0), (i0 + 1, j0), (i0 + 1, j0 + 1)]
            lam = [1.0 - s, s - q, q]
        else:        # upper triangle [(i,j), (i+1,j+1), (i,j+1)]
            verts = [(i0, j0), (i0 + 1, j0 + 1), (i0, j0 + 1)]
            lam = [1.0 - q, s, q - s]
        for (vi, vj), w in zip(verts, lam):
            if w == 0.0:
                continue
            c = cidx[vi * ntc + (vj % ntc)]
            if c < 0:          # Dirichlet coarse node: value 0
                continue
            rows.append(fidx[node])
            cols.append(c)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_interior, coarse.n_interior))


def restriction(P, kind="normalized"):
    """R_s from P_s: 'normalized' = D^{-1} P^T, 'transpose' = P^T."""
    Rt = P.T.tocsr()
    if kind == "transpose":
        return Rt
    if kind == "normalized":
        d = np.asarray(Rt.sum(axis=1)).ravel()
        return sp.diags(1.0 / d) @ Rt
    raise ValueError(kind)


def injection(fine, coarse):
    """R_inj: coarse interior node (i, j) takes fine node (2i, 2j)."""
    check_nested(fine, coarse)
    fidx = _interior_index(fine)
    rows, cols = [], []
    for c, node in enumerate(coarse.interior_nodes()):
        i, j = divmod(int(node), coarse.n_theta)
        rows.append(c)
        cols.append(fidx[(2 * i) * fine.n_theta + 2 * j])
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)),
                         shape=(coarse.n_interior, fine.n_interior))
