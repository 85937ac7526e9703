"""GPU parity of the batched propagator Phi (eq. 2, eq. 8) against the oracle's
direct sparse solve, through the C ABI (phi_step)."""

import numpy as np
import pytest

from workload import config, polar_mesh
from workload.configs import LevelSpec
from oracle.stepping import Level, sequential

pytestmark = pytest.mark.gpu

PHI_TOL = 1e-10          # relative 2-norm error per column (FP64 Phi)


def _solver(cfg, **kw):
    from paper_1912_03106_amd.solver import Solver
    return Solver(cfg, **kw)


def _col_err(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.fixture(scope="module")
def cfg1_pair():
    cfg = config("cfg1")
    s = _solver(cfg, pcg_tol=1e-13)
    lev = Level(polar_mesh(16, 128), cfg.dt, cfg.source)
    U = sequential(lev, np.zeros(lev.n), 200)
    return cfg, s, lev, U


@pytest.fixture(scope="module")
def solvers_by_kernel(cfg1_pair):
    """phi_step with each batched-CG kernel family forced: general sparse
    rows (1) and the diagonal window of the periodic polar stencil (2)."""
    cfg = cfg1_pair[0]
    return {k: _solver(cfg, pcg_tol=1e-13, pcg_kernel=k) for k in (1, 2)}


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("B", [1, 63, 64, 65, 200])
def test_phi_matches_direct_solve(cfg1_pair, solvers_by_kernel, B, kernel):
    cfg, _, lev, U = cfg1_pair
    s = solvers_by_kernel[kernel]
    print(f"phi parity 16x128 B={B} kernel={kernel}", flush=True)
    rng = np.random.default_rng(B)
    i_from = rng.integers(0, cfg.n_steps - 1, size=B)
    # realistic states (a trajectory) plus a perturbation
    u_prev = U[rng.integers(1, U.shape[0], size=B)] + 1e-4 * rng.standard_normal((B, lev.n))
    got = s.phi(0, u_prev, i_from)
    ref = lev.phi(u_prev, i_from)
    err = _col_err(got, ref)
    assert err.max() <= PHI_TOL, err.max()


def test_phi_coarse_level_step(cfg1_pair):
    """Level 1 of the two-level hierarchy uses dt_1 = m dt (re-discretisation)."""
    cfg, s, _, U = cfg1_pair
    lev1 = Level(polar_mesh(16, 128), cfg.level_dt(1), cfg.source)
    rng = np.random.default_rng(7)
    u_prev = U[rng.integers(1, U.shape[0], size=10)]
    i_from = rng.integers(0, cfg.level_steps(1) - 1, size=10)
    err = _col_err(s.phi(1, u_prev, i_from), lev1.phi(u_prev, i_from))
    assert err.max() <= PHI_TOL, err.max()


def test_phi_is_deterministic(cfg1_pair):
    cfg, s, lev, U = cfg1_pair
    rng = np.random.default_rng(3)
    u_prev = U[rng.integers(1, U.shape[0], size=70)]
    i_from = rng.integers(0, 1000, size=70)
    a = s.phi(0, u_prev, i_from)
    b = s.phi(0, u_prev, i_from)
    assert np.array_equal(a, b)


def test_phi_edge_cases(cfg1_pair):
    cfg, s, lev, U = cfg1_pair
    from paper_1912_03106_amd import MgritError
    # zero state at a time where every source is active equals the magnetostatic-with-mass solve
    out = s.phi(0, np.zeros((2, lev.n)), [0, 511])
    ref = lev.phi(np.zeros((2, lev.n)), [0, 511])
    assert _col_err(out, ref).max() <= PHI_TOL
    with pytest.raises(MgritError) as e:
        s.phi(5, np.zeros((1, lev.n)), [0])
    assert e.value.name == "INVALID_ARGUMENT"


def test_phi_full_size_sampled_columns():
    """The 64 x 512 level of the large linear workload (n = 32,256, dt = 0.02/16384),
    on sampled columns the oracle solves one by one."""
    print("phi parity 64x512 sampled", flush=True)
    cfg = config("cfg2")
    cfg.meshes = [LevelSpec(64, 512), LevelSpec(32, 256)]
    s = _solver(cfg, pcg_tol=1e-13, m=16)
    lev = Level(polar_mesh(64, 512), cfg.dt, cfg.source)
    U = sequential(lev, np.zeros(lev.n), 24)
    rng = np.random.default_rng(11)
    i_from = np.array([3, 100, 2047, 5000, 9999, 16382, 12, 777])
    u_prev = U[rng.integers(5, 25, size=8)]
    got = s.phi(0, u_prev, i_from)
    ref = lev.phi(u_prev, i_from)
    err = _col_err(got, ref)
    assert err.max() <= PHI_TOL, err


def test_phi_fp32_refinement_matches_direct_solve(cfg1_pair):
    """FP32 inner PCG with FP64 iterative refinement reaches the FP64 accuracy."""
    cfg, _, lev, U = cfg1_pair
    print("phi parity FP32+IR 16x128", flush=True)
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, pcg_tol=1e-13, precision=_abi.FP32_IR, ir_inner_tol=1e-4)
    rng = np.random.default_rng(21)
    B = 97
    i_from = rng.integers(0, cfg.n_steps - 1, size=B)
    u_prev = U[rng.integers(1, U.shape[0], size=B)] + 1e-4 * rng.standard_normal((B, lev.n))
    err = _col_err(s.phi(0, u_prev, i_from), lev.phi(u_prev, i_from))
    assert err.max() <= PHI_TOL, err.max()


def test_phi_fp32_refinement_full_size():
    print("phi parity FP32+IR 64x512 sampled", flush=True)
    from paper_1912_03106_amd import _abi
    cfg = config("cfg3")
    cfg.meshes = [LevelSpec(64, 512), LevelSpec(32, 256)]
    s = _solver(cfg, pcg_tol=1e-13, precision=_abi.FP32_IR, ir_inner_tol=1e-4)
    lev = Level(polar_mesh(64, 512), cfg.dt, cfg.source)
    U = sequential(lev, np.zeros(lev.n), 12)
    i_from = np.array([3, 4095, 8191, 16000])
    u_prev = U[[4, 7, 9, 12]]
    err = _col_err(s.phi(0, u_prev, i_from), lev.phi(u_prev, i_from))
    assert err.max() <= PHI_TOL, err


def test_phi_full_size_compaction_identical():
    """A 600-column batched Phi on the 64x512 level with warm starts of
    different quality: compacting the iterating columns gives the same bits."""
    print("phi 64x512 compaction", flush=True)
    cfg = config("cfg2")
    lev = Level(polar_mesh(64, 512), cfg.dt, cfg.source)
    U = sequential(lev, np.zeros(lev.n), 6)
    rng = np.random.default_rng(9)
    B = 600
    u_prev = U[rng.integers(1, 7, size=B)] * rng.uniform(0.2, 3.0, size=(B, 1))
    i_from = rng.integers(0, cfg.n_steps - 1, size=B)
    outs = []
    for k in (0, 64):
        s = _solver(cfg, compact_columns=k, pcg_tol=1e-12)
        outs.append(s.phi(0, u_prev, i_from))
        s.close()
    assert np.array_equal(outs[0], outs[1])
    pick = [0, 299, 599]
    err = _col_err(outs[1][pick], lev.phi(u_prev[pick], i_from[pick]))
    assert err.max() <= PHI_TOL, err


@pytest.mark.parametrize("B", [1, 64, 100, 1030])
def test_phi_intermediate_level_stored_inverse(B):
    """An intermediate level that steps by its stored inverse (the product
    X = A^{-1} B on the FP64 matrix cores, k split over work-groups for narrow
    batches): the 32x256 level 1 of the large workload against the direct
    solve, batches of 1, 64 (the relaxation sweeps), 100 and 1030 (ragged
    tiles) columns."""
    print(f"phi stored inverse 32x256 B={B}", flush=True)
    cfg = config("cfg2")
    s = _solver(cfg, pcg_tol=1e-13, coarse_inverse=2)
    lev = Level(polar_mesh(32, 256), cfg.level_dt(1), cfg.source)
    U = sequential(lev, np.zeros(lev.n), 30)
    rng = np.random.default_rng(B)
    i_from = rng.integers(0, cfg.level_steps(1) - 1, size=B)
    u_prev = U[rng.integers(1, 31, size=B)] * rng.uniform(0.5, 1.5, size=(B, 1))
    err = _col_err(s.phi(1, u_prev, i_from), lev.phi(u_prev, i_from))
    assert err.max() <= PHI_TOL, err.max()
