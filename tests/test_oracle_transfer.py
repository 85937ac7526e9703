"""Pins of the oracle's spatial transfers (Sec. 2.2, Sec. 3.4): nodal
interpolation must be exact on linear functions, coincide with injection at
coincident nodes, and the normalised restriction must preserve constants."""

import numpy as np
import pytest

from workload import polar_mesh
from oracle import transfer


@pytest.fixture(scope="module")
def pair():
    fine, coarse = polar_mesh(16, 64), polar_mesh(8, 32)
    return fine, coarse, transfer.prolongation(fine, coarse)


def test_injection_after_prolongation_is_identity(pair):
    fine, coarse, P = pair
    Ri = transfer.injection(fine, coarse)
    I = (Ri @ P).toarray()
    assert np.array_equal(I, np.eye(coarse.n_interior))


def test_prolongation_reproduces_logical_linear_functions(pair):
    """A function linear in the logical (i, j) coordinates is interpolated
    exactly wherever its coarse stencil avoids the boundary and the theta wrap."""
    fine, coarse, P = pair
    a, b, c = 0.7, -1.3, 0.25
    ci, cj = np.divmod(coarse.interior_nodes(), coarse.n_theta)
    fI, fJ = np.divmod(fine.interior_nodes(), fine.n_theta)
    uc = a + b * ci + c * cj
    uf = P @ uc
    ok = (fI >= 2) & (fI <= fine.n_r - 2) & (fJ <= fine.n_theta - 2)
    ref = a + b * fI / 2.0 + c * fJ / 2.0
    assert np.abs(uf[ok] - ref[ok]).max() < 1e-13
    assert ok.sum() > fine.n_interior // 2


def test_prolongation_row_structure(pair):
    fine, coarse, P = pair
    fI, fJ = np.divmod(fine.interior_nodes(), fine.n_theta)
    nnz = np.diff(P.indptr)
    even = (fI % 2 == 0) & (fJ % 2 == 0)
    assert (nnz[even] == 1).all()
    inner = (fI >= 2) & (fI <= fine.n_r - 2)
    assert (nnz[~even & inner] == 2).all()
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel()[inner], 1.0)


def test_normalized_restriction_preserves_constants(pair):
    fine, coarse, P = pair
    R = transfer.restriction(P)
    assert np.allclose(R @ np.ones(fine.n_interior), 1.0, rtol=0, atol=1e-14)
    # interior rows: the coincident node (weight 1) and six neighbours (1/2) over 4
    row = R.getrow(coarse.n_theta * 3 + 5)
    assert sorted(np.round(row.data * 8).astype(int).tolist()) == [1, 1, 1, 1, 1, 1, 2]


def test_not_nested_is_rejected():
    with pytest.raises(ValueError):
        transfer.prolongation(polar_mesh(16, 64), polar_mesh(8, 16))
