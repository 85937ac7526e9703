"""GPU batched Newton (saturating iron, Sec. 3.1 / Sec. 5) against the oracle's
Newton with direct solves, through the C ABI."""

import numpy as np
import pytest

from workload import config, polar_mesh, Source, BHLaw
from workload.configs import LevelSpec
from oracle.stepping import Level, sequential
from oracle.problem import build
from oracle import mgrit

pytestmark = pytest.mark.gpu

PHI_TOL = 1e-10
# Twice the default current density and no start-up ramp: over the first
# quarter period the oracle's damped Newton takes 2 to 11 iterations per step
# on 16x128, with shortened steps in about half of them
STRONG = Source(J0=2e7)
MAXIT = 16          # oracle Newton steps
GPU_MAXIT = 24      # GPU Newton steps (inexact inner solves)
# The oracle's Newton stops at ||R|| <= tol ||R(u_prev)||; the solution error
# can be ~10x that, so the Phi comparisons run the oracle two digits tighter
# than the 1e-10 they check.
ORACLE_TOL = 1e-12


def _solver(cfg, **kw):
    from paper_1912_03106_amd.solver import Solver
    return Solver(cfg, **kw)


def _col_err(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _small_cfg(**kw):
    base = dict(meshes=[LevelSpec(16, 128), LevelSpec(16, 128)], n_steps=256, m=16,
                t_final=0.005, source=STRONG, newton_maxit=MAXIT, newton_tol=ORACLE_TOL)
    base.update(kw)
    return config("cfg4", **base)


@pytest.fixture(scope="module")
def nl_pair():
    cfg = _small_cfg()
    lev = Level(polar_mesh(16, 128), cfg.dt, cfg.source, bh=cfg.bh, newton_maxit=MAXIT,
                newton_tol=ORACLE_TOL)
    U = sequential(lev, np.zeros(lev.n), 160)
    assert min(lev.newton_lambdas) < 1.0         # damping was needed on the way
    return cfg, lev, U


@pytest.mark.parametrize("B", [1, 64, 97])
def test_newton_phi_fp64_matches_oracle(nl_pair, B):
    print(f"newton phi fp64 B={B}", flush=True)
    cfg, lev, U = nl_pair
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP64, ir_inner_tol=1e-6, newton_tol=1e-12,
                newton_max_iter=GPU_MAXIT)
    rng = np.random.default_rng(B)
    i_from = rng.integers(0, cfg.n_steps - 1, size=B)
    u_prev = U[rng.integers(5, U.shape[0], size=B)]
    got = s.phi(0, u_prev, i_from)
    ref = lev.phi(u_prev, i_from)
    assert max(lev.newton_iters[-B:]) >= 2          # genuinely nonlinear steps
    err = _col_err(got, ref)
    assert err.max() <= PHI_TOL, err.max()


def test_newton_phi_fp32_inner_matches_oracle(nl_pair):
    print("newton phi fp32 inner", flush=True)
    cfg, lev, U = nl_pair
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP32_IR, ir_inner_tol=1e-5, newton_tol=1e-12,
                newton_max_iter=GPU_MAXIT)
    rng = np.random.default_rng(5)
    i_from = rng.integers(0, cfg.n_steps - 1, size=65)
    u_prev = U[rng.integers(5, U.shape[0], size=65)]
    err = _col_err(s.phi(0, u_prev, i_from), lev.phi(u_prev, i_from))
    assert err.max() <= PHI_TOL, err.max()


def test_newton_phi_full_size_sampled_columns():
    """The 64 x 512 level of the nonlinear workload (dt = 0.02/32768)."""
    print("newton phi 64x512 sampled", flush=True)
    cfg = config("cfg4", source=STRONG, newton_maxit=MAXIT)
    cfg.meshes = [LevelSpec(64, 512), LevelSpec(32, 256)]
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP64, ir_inner_tol=1e-6, newton_tol=1e-12,
                newton_max_iter=GPU_MAXIT)
    lev = Level(polar_mesh(64, 512), cfg.dt, cfg.source, bh=cfg.bh, newton_maxit=MAXIT,
                newton_tol=ORACLE_TOL)
    U = sequential(lev, np.zeros(lev.n), 6)
    assert max(lev.newton_iters) >= 4
    i_from = np.array([5, 8191, 20000, 32760])
    u_prev = U[[3, 4, 5, 6]]
    err = _col_err(s.phi(0, u_prev, i_from), lev.phi(u_prev, i_from))
    assert err.max() <= PHI_TOL, err


@pytest.mark.parametrize("seq_kernel", [1, 2])
def test_newton_seq_solve_matches_oracle(nl_pair, seq_kernel):
    """Sequential damped-Newton stepping in one persistent work-group (the
    whole sweep on the device, seq_kernel = 1) and with the batched kernels
    step by step (seq_kernel = 2) against the oracle."""
    print(f"newton seq kernel {seq_kernel}", flush=True)
    cfg, lev, _ = nl_pair
    cfg = _small_cfg(n_steps=64, t_final=64 * cfg.dt)
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP64, ir_inner_tol=1e-6, newton_tol=1e-12,
                newton_max_iter=GPU_MAXIT, seq_kernel=seq_kernel)
    U, st = s.seq_solve()
    assert st["newton_sweeps"][0] > 64
    U_ref = sequential(lev, np.zeros(lev.n), 64)
    err = np.linalg.norm(U - U_ref, axis=1)[1:] / np.linalg.norm(U_ref, axis=1)[1:]
    assert err.max() <= PHI_TOL * 10, err.max()


def test_newton_mgrit_two_level_matches_oracle():
    print("newton mgrit two-level", flush=True)
    cfg = _small_cfg()
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    _, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=cfg.mgrit_tol, maxit=2)
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP32_IR, ir_inner_tol=1e-5, newton_tol=1e-11,
                newton_max_iter=GPU_MAXIT, pcg_tol=1e-12)
    U, st = s.solve()
    assert st["converged"]
    for a, b in zip(st["rho"][:3], hist[:3]):
        assert abs(a - b) <= 1e-8 * hist[0], (a, b)
    assert _rel(U, U_seq) <= 1e-7
    assert sum(st["newton_sweeps"]) > 0


def test_newton_cap_is_reported(nl_pair):
    cfg, lev, U = nl_pair
    from paper_1912_03106_amd import MgritError, _abi
    s = _solver(cfg, precision=_abi.FP64, newton_max_iter=1, newton_tol=1e-14)
    with pytest.raises(MgritError) as e:
        s.phi(0, U[[20, 30]], [10, 20])
    assert e.value.name == "NEWTON_NOT_CONVERGED"


def test_newton_graph_replay_matches_eager(nl_pair):
    print("newton graphs vs eager", flush=True)
    cfg, lev, U = nl_pair
    from paper_1912_03106_amd import _abi
    rng = np.random.default_rng(11)
    i_from = rng.integers(0, cfg.n_steps - 1, size=40)
    u_prev = U[rng.integers(5, U.shape[0], size=40)]
    out = [_solver(cfg, precision=_abi.FP32_IR, newton_tol=1e-12, newton_max_iter=GPU_MAXIT,
                   use_graphs=g).phi(0, u_prev, i_from) for g in (0, 1)]
    assert np.array_equal(out[0], out[1])


def test_damped_newton_hard_steps_match_oracle():
    """From rest under a current density so high that a full Newton step
    overflows the reluctivity: both sides damp their steps (down to 1/32 here)
    and must land on the same solution; plain Newton fails on the GPU too."""
    print("newton damped hard steps", flush=True)
    from paper_1912_03106_amd import MgritError, _abi
    cfg = _small_cfg(source=Source(J0=3e8), newton_maxit=30)
    lev = Level(polar_mesh(16, 128), cfg.dt, cfg.source, bh=cfg.bh, newton_maxit=30,
                newton_tol=ORACLE_TOL)
    i_from = np.array([0, 3, 50, 100, 200, 255])
    u_prev = np.zeros((len(i_from), lev.n))
    ref = lev.phi(u_prev, i_from)
    assert min(lev.newton_lambdas) < 0.1
    s = _solver(cfg, precision=_abi.FP64, ir_inner_tol=1e-6, newton_tol=1e-12, newton_max_iter=40)
    err = _col_err(s.phi(0, u_prev, i_from), ref)
    assert err.max() <= PHI_TOL, err
    plain = _solver(cfg, precision=_abi.FP64, ir_inner_tol=1e-6, newton_tol=1e-12,
                    newton_max_iter=40, newton_halvings=0)
    with pytest.raises(MgritError) as e:
        plain.phi(0, u_prev, i_from)
    assert e.value.name in ("NONFINITE", "NEWTON_NOT_CONVERGED")


def test_newton_early_stopped_relaxation_reaches_the_same_solution():
    """Level-0 relaxation Newton solves stopped at eta times their warm-start
    residual: MGRIT still converges to the sequential solution."""
    print("newton mgrit early stop", flush=True)
    cfg = _small_cfg()
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP32_IR, ir_inner_tol=1e-5, newton_tol=1e-11,
                newton_max_iter=GPU_MAXIT, pcg_tol=1e-12, pcg_tol_eta=1e-3)
    U, st = s.solve()
    assert st["converged"]
    assert _rel(U, U_seq) <= 1e-7


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_newton_jacobian_layouts_agree(nl_pair, precision):
    """The Jacobian stored by stencil offset (upper half of the symmetric
    matrix, diagonal-window CG passes) and on the general sparse rows
    (pcg_kernel = 1): both reach the oracle's Newton solution."""
    print(f"newton jacobian layouts {precision}", flush=True)
    cfg, lev, U = nl_pair
    from paper_1912_03106_amd import _abi
    prec = _abi.FP64 if precision == "fp64" else _abi.FP32_IR
    rng = np.random.default_rng(17)
    B = 70
    i_from = rng.integers(0, cfg.n_steps - 1, size=B)
    u_prev = U[rng.integers(5, U.shape[0], size=B)]
    ref = lev.phi(u_prev, i_from)
    outs = []
    for kernel in (0, 1):
        s = _solver(cfg, precision=prec, ir_inner_tol=1e-6, newton_tol=1e-12, newton_max_iter=GPU_MAXIT,
                    pcg_kernel=kernel)
        outs.append(s.phi(0, u_prev, i_from))
        s.close()
    for out in outs:
        assert _col_err(out, ref).max() <= PHI_TOL


@pytest.mark.parametrize("persistent", [-1, 1])
def test_newton_mgrit_coarsest_persistent_and_batched_agree(persistent):
    """The coarsest level's sequential Newton sweep in one persistent
    work-group or with the batched kernels step by step: the same history
    (to the Newton tolerance) and the sequential solution."""
    print(f"newton mgrit coarsest persistent {persistent}", flush=True)
    cfg = _small_cfg()
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    _, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=cfg.mgrit_tol, maxit=2)
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, precision=_abi.FP32_IR, ir_inner_tol=1e-5, newton_tol=1e-11,
                newton_max_iter=GPU_MAXIT, pcg_tol=1e-12, coarse_persistent=persistent)
    U, st = s.solve()
    assert st["converged"]
    for a, b in zip(st["rho"][:3], hist[:3]):
        assert abs(a - b) <= 1e-8 * hist[0], (a, b)
    assert _rel(U, U_seq) <= 1e-7
    assert st["newton_sweeps"][1] > 0


@pytest.mark.parametrize("B", [1, 17, 200])
def test_newton_coarse_level_narrow_persistent_matches_oracle(nl_pair, B):
    """Narrow batches on a coarse level (dt_1 = m dt): one persistent
    work-group per column runs the whole damped Newton solve
    (coarse_persistent = 1) or the batched kernels do (the default); both
    reach the oracle's Newton solution."""
    print(f"newton level-1 narrow persistent B={B}", flush=True)
    cfg, _, U = nl_pair
    lev1 = Level(polar_mesh(16, 128), cfg.level_dt(1), cfg.source, bh=cfg.bh, newton_maxit=MAXIT,
                 newton_tol=ORACLE_TOL)
    rng = np.random.default_rng(100 + B)
    i_from = rng.integers(0, cfg.level_steps(1) - 1, size=B)
    u_prev = U[rng.integers(5, U.shape[0], size=B)]
    ref = lev1.phi(u_prev, i_from)
    from paper_1912_03106_amd import _abi
    for persistent in (1, 0):
        s = _solver(cfg, precision=_abi.FP64, ir_inner_tol=1e-6, newton_tol=1e-12,
                    newton_max_iter=GPU_MAXIT, coarse_persistent=persistent)
        err = _col_err(s.phi(1, u_prev, i_from), ref)
        s.close()
        assert err.max() <= PHI_TOL, (persistent, err.max())
