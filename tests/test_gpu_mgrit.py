"""GPU FAS-MGRIT and GPU sequential stepping against the oracle (Algorithm 1,
Sec. 2.1, Sec. 2.2), through the C ABI."""

import numpy as np
import pytest

from workload import config
from workload.configs import LevelSpec
from oracle.problem import build
from oracle import mgrit, stepping

pytestmark = pytest.mark.gpu

SEQ_TOL = 1e-10     # GPU sequential stepping vs the direct-solve oracle
MGRIT_GATE = 1e-7   # ||U - U_seq|| / ||U_seq|| after MGRIT stops at rho <= 1e-8 rho_0


def _solver(cfg, **kw):
    from paper_1912_03106_amd.solver import Solver
    return Solver(cfg, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def cfg1_oracle():
    cfg = config("cfg1")
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    U_mg, hist, conv = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=cfg.mgrit_tol, maxit=40)
    assert conv
    return cfg, U_seq, U_mg, hist


@pytest.mark.parametrize("seq_kernel", [1, 2, 3])
def test_seq_solve_matches_oracle(cfg1_oracle, seq_kernel):
    """GPU sequential stepping (one work-group, the cooperative grid, or the
    level's stored inverse streamed once per step) vs the oracle's
    direct-solve stepping."""
    print(f"seq cfg1 kernel {seq_kernel}", flush=True)
    cfg, U_seq, _, _ = cfg1_oracle
    s = _solver(cfg, pcg_tol=1e-13, seq_kernel=seq_kernel)
    U, st = s.seq_solve()
    assert U.shape == U_seq.shape
    err = np.linalg.norm(U - U_seq, axis=1)[1:] / np.linalg.norm(U_seq, axis=1)[1:]
    assert err.max() <= SEQ_TOL, err.max()
    if seq_kernel == 3:
        # the inverse built for the sequential solve leaves the handle's MGRIT
        # solve on its batched level-0 solves
        U2, st2 = s.solve()
        assert st2["converged"] and st2["pcg_sweeps"][0] > 0
        assert _rel(U2, U_seq) <= MGRIT_GATE


def test_mgrit_two_level_matches_oracle(cfg1_oracle):
    """Linear 16x128 machine, 1024 steps, two-level FCF, m = 16, no spatial coarsening."""
    print("mgrit cfg1", flush=True)
    cfg, U_seq, U_mg, hist = cfg1_oracle
    s = _solver(cfg, pcg_tol=1e-12)
    U, st = s.solve()
    assert st["converged"]
    # same iteration count as the textbook oracle (round-off may move the last one)
    assert abs(len(st["rho"]) - len(hist)) <= 1, (st["rho"], hist)
    # residual histories agree, on the scale of rho_0, down to the MGRIT tolerance
    for a, b in zip(st["rho"], hist):
        assert abs(a - b) <= 1e-9 * hist[0], (a, b)
    assert _rel(U, U_seq) <= MGRIT_GATE
    assert _rel(U, U_mg) <= MGRIT_GATE
    # and at every time point (the oracle's own MGRIT iterate is within
    # 8e-10 of sequential stepping at every point)
    for ref in (U_seq, U_mg):
        err = np.linalg.norm(U - ref, axis=1)[1:] / np.linalg.norm(ref, axis=1)[1:]
        assert err.max() <= 1e-8, (int(np.argmax(err)), err.max())
    assert st["rho"][-1] <= cfg.mgrit_tol * st["rho"][0]


def test_mgrit_exact_after_nt_over_2m_fcf(cfg1_oracle):
    """FCF reaches the sequential solution after N_t/(2m) iterations (Sec. 2.1)."""
    cfg, U_seq, _, _ = cfg1_oracle
    s = _solver(cfg, pcg_tol=1e-13, tol=0.0, max_iter=32)
    U, st = s.solve(raise_on_stall=False)
    # it may stop earlier: once every C-point satisfies Phi to the solver
    # tolerance, the warm-started residual solve returns rho = 0 exactly
    assert st["iterations"] <= 32
    assert _rel(U, U_seq) <= 1e-10


def _sc_cfg():
    cfg = config("cfg1")
    cfg.meshes = [LevelSpec(32, 256), LevelSpec(16, 128), LevelSpec(8, 64)]
    cfg.n_steps, cfg.m = 1024, 16
    return cfg


def test_mgrit_three_level_spatial_coarsening_matches_oracle():
    """Three-level V-cycle, direct spatial coarsening 32x256 -> 16x128 -> 8x64."""
    print("mgrit 3-level SC", flush=True)
    cfg = _sc_cfg()
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    s = _solver(cfg, pcg_tol=1e-12)
    U, st = s.solve()
    assert st["converged"]
    assert _rel(U, U_seq) <= MGRIT_GATE
    # iteration count of the textbook algorithm on this problem (oracle: 11)
    _, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=cfg.mgrit_tol, maxit=3)
    for a, b in zip(st["rho"][:4], hist[:4]):
        assert abs(a - b) <= 1e-9 * hist[0], (a, b)
    assert abs(len(st["rho"]) - 11) <= 1


def test_mgrit_failure_modes(cfg1_oracle):
    cfg, _, _, _ = cfg1_oracle
    from paper_1912_03106_amd import MgritError
    s = _solver(cfg, pcg_max_iter=1)
    with pytest.raises(MgritError) as e:
        s.solve()
    assert e.value.name == "PCG_NOT_CONVERGED"
    s = _solver(cfg, max_iter=1)
    with pytest.raises(MgritError) as e:
        s.solve()
    assert e.value.name == "NOT_CONVERGED"
    s = _solver(cfg)
    guess = np.zeros((cfg.n_steps + 1, s.n0))
    guess[5, 3] = np.nan          # an F-point: F-relaxation overwrites it, harmless
    U, st = s.solve(u_init=guess)
    assert st["converged"] and np.isfinite(U).all()
    guess[5 * cfg.m, 3] = np.nan  # a C-point feeds the first F-relaxation
    with pytest.raises(MgritError) as e:
        s.solve(u_init=guess)
    assert e.value.name == "NONFINITE"


def test_mgrit_fp32_refinement_random_guess_matches_oracle(cfg1_oracle):
    """FP32 inner solves + FP64 refinement, seeded U(-1e-3, 1e-3) initial guess:
    the same gate against the FP64 sequential solution."""
    print("mgrit cfg1 FP32+IR random guess", flush=True)
    cfg, U_seq, _, _ = cfg1_oracle
    from paper_1912_03106_amd import _abi
    s = _solver(cfg, pcg_tol=1e-12, precision=_abi.FP32_IR, ir_inner_tol=1e-4)
    rng = np.random.default_rng(3)
    guess = np.zeros((cfg.n_steps + 1, s.n0))
    guess[1:] = rng.uniform(-1e-3, 1e-3, size=(cfg.n_steps, s.n0))
    U, st = s.solve(u_init=guess)
    assert st["converged"]
    assert _rel(U, U_seq) <= MGRIT_GATE


@pytest.mark.parametrize("kernel", [1, 2])
def test_mgrit_kernel_families_agree(cfg1_oracle, kernel):
    """The two batched-CG kernel families give the same MGRIT run."""
    cfg, U_seq, _, hist = cfg1_oracle
    s = _solver(cfg, pcg_tol=1e-12, pcg_kernel=kernel)
    U, st = s.solve()
    assert st["converged"] and abs(len(st["rho"]) - len(hist)) <= 1
    assert _rel(U, U_seq) <= MGRIT_GATE


def test_diagonal_window_rejects_non_polar_mesh():
    from paper_1912_03106_amd import MgritError
    from workload import polar_mesh
    cfg = config("cfg1")
    meshes = [polar_mesh(16, 128), polar_mesh(16, 128)]
    for m in meshes:
        m.n_r = 0
        m.n_theta = 0
    with pytest.raises(MgritError) as e:
        _solver(cfg, meshes=meshes, pcg_kernel=2)
    assert e.value.name == "UNSUPPORTED"


@pytest.mark.parametrize("coarse_inverse", [0, 1, 2])
def test_mgrit_coarsest_solver_variants_agree(cfg1_oracle, coarse_inverse):
    """Coarse levels stepped by PCG or by stored inverses (coarsest only, or
    every coarse level through FP64 GEMMs): same iterates."""
    cfg, U_seq, _, hist = cfg1_oracle
    s = _solver(cfg, pcg_tol=1e-12, coarse_inverse=coarse_inverse)
    U, st = s.solve()
    assert st["converged"] and abs(len(st["rho"]) - len(hist)) <= 1
    for a, b in zip(st["rho"], hist):
        assert abs(a - b) <= 1e-9 * hist[0]
    assert _rel(U, U_seq) <= MGRIT_GATE


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_graph_replay_matches_eager_launches(cfg1_oracle, precision):
    """Check intervals of CG iterations replayed from captured hipGraphs give
    bit-identical iterates to launching every kernel from the host."""
    print(f"graphs vs eager {precision}", flush=True)
    from paper_1912_03106_amd import _abi
    cfg, U_seq, _, hist = cfg1_oracle
    prec = _abi.FP64 if precision == "fp64" else _abi.FP32_IR
    runs = []
    for g in (0, 1):
        s = _solver(cfg, pcg_tol=1e-12, precision=prec, use_graphs=g)
        U, st = s.solve()
        U2, st2 = s.solve()          # replays graphs captured by the first solve
        assert np.array_equal(U, U2) and st["rho"] == st2["rho"]
        runs.append((U, st))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1]["rho"] == runs[1][1]["rho"]
    assert _rel(runs[1][0], U_seq) <= MGRIT_GATE


def test_seq_solve_with_startup_ramp_matches_oracle():
    """The start-up ramp of the nonlinear model's source, on the linear machine."""
    print("seq cfg1 ramp", flush=True)
    from workload import Source
    cfg = config("cfg1", source=Source(ramp_periods=2.0), n_steps=256, t_final=0.005)
    H, _ = build(cfg)
    U_ref = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), cfg.n_steps)
    U, _ = _solver(cfg, pcg_tol=1e-13).seq_solve()
    err = np.linalg.norm(U - U_ref, axis=1)[1:] / np.linalg.norm(U_ref, axis=1)[1:]
    assert err.max() <= SEQ_TOL, err.max()


@pytest.mark.parametrize("variant", ["fp64_eta", "fp32ir_eta_coarse_fp64", "fp64_delta_start",
                                     "fp32ir_delta_start"])
def test_early_stopped_relaxation_reaches_the_same_solution(variant):
    """Level-0 relaxation solves stopped at max(pcg_tol ||b||, eta ||r_0||)
    (the coarse levels keep pcg_tol): the same fixed point, within one or two
    iterations of the strict solves.  The delta-start variants also start the
    F-relaxation solves from the previous iterate plus the change of their
    input (warm_start = 2) and stop the C-point residual solves at 1e-4 of
    their warm-start residual."""
    print(f"mgrit early stop {variant}", flush=True)
    from paper_1912_03106_amd import _abi
    cfg = _sc_cfg()
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    kw = dict(pcg_tol=1e-12, pcg_tol_eta=1e-3)
    if variant.endswith("delta_start"):
        kw.update(pcg_tol_eta=3e-3, warm_start=2, residual_eta=1e-4)
    if variant.startswith("fp32ir"):
        kw.update(precision=_abi.FP32_IR, precision_coarse=_abi.FP64)
    U, st = _solver(cfg, **kw).solve()
    assert st["converged"]
    assert len(st["rho"]) <= 11 + 2
    assert _rel(U, U_seq) <= MGRIT_GATE


@pytest.mark.parametrize("narrow", [-1, 16])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_column_compaction_gives_identical_iterates(cfg1_oracle, precision, narrow):
    """Gathering the still-iterating CG columns densely (here whenever one
    column would drop out) leaves every column's arithmetic unchanged, also
    when the passes switch to 16-row work-groups once at most 128 columns
    iterate (narrow = 16; on this 64-interval workload from the first check)."""
    print(f"compaction {precision} narrow {narrow}", flush=True)
    from paper_1912_03106_amd import _abi
    cfg, U_seq, _, _ = cfg1_oracle
    prec = _abi.FP64 if precision == "fp64" else _abi.FP32_IR
    out = []
    for k in (0, 1):
        U, st = _solver(cfg, pcg_tol=1e-12, precision=prec, compact_columns=k,
                        pcg_tol_eta=1e-3, pcg_rows_narrow=narrow).solve()
        out.append((U, st))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1]["rho"] == out[1][1]["rho"]
    assert _rel(out[1][0], U_seq) <= MGRIT_GATE


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_prefetch_depth_gives_identical_iterates(precision):
    """The diagonal-window CG passes load their window rows 1, 2 or 4 rows
    ahead; a row's arithmetic is the same, so the iterates are bitwise equal.
    On the 16x126 mesh n = 1890, so with 16-row walks the last wave has 2
    rows (a partly filled ring), and column compaction runs as well."""
    print(f"prefetch depth {precision}", flush=True)
    from paper_1912_03106_amd import _abi
    cfg = config("cfg1", meshes=[LevelSpec(16, 126), LevelSpec(16, 126)])
    H, _ = build(cfg)
    U_seq = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), cfg.n_steps)
    prec = _abi.FP64 if precision == "fp64" else _abi.FP32_IR
    out = []
    for depth in (1, 2, 4):
        s = _solver(cfg, pcg_tol=1e-12, precision=prec, pcg_kernel=2, pcg_prefetch=depth,
                    compact_columns=1, pcg_tol_eta=1e-3)
        assert s.kernel_shape(0)[2:4] == (2, depth)
        out.append(s.solve())
        s.close()
    for U, st in out[1:]:
        assert np.array_equal(U, out[0][0])
        assert st["rho"] == out[0][1]["rho"]
    assert out[0][1]["converged"]
    assert _rel(out[0][0], U_seq) <= MGRIT_GATE


def test_pinned_kernel_shape_is_used_and_matches_oracle():
    """Rows per work-group, columns per lane, prefetch depth and narrow-set
    rows pinned instead of autotuned (the hardware-counter runs): the level
    reports exactly that shape and MGRIT still reaches the sequential solution."""
    print("pinned kernel shape", flush=True)
    cfg = config("cfg1", meshes=[LevelSpec(16, 126), LevelSpec(16, 126)])
    H, _ = build(cfg)
    U_seq = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), cfg.n_steps)
    s = _solver(cfg, pcg_tol=1e-12, pcg_kernel=2, pcg_rows_per_block=32, pcg_cols_per_lane=2,
                pcg_prefetch=2, pcg_rows_narrow=16)
    assert s.kernel_shape(0) == (32, 2, 2, 2, 16)
    U, st = s.solve()
    s.close()
    assert st["converged"]
    assert _rel(U, U_seq) <= MGRIT_GATE


@pytest.mark.parametrize("bad", [dict(pcg_prefetch=3), dict(warm_start=3), dict(residual_eta=1.0),
                                 dict(residual_eta=-1e-3), dict(pcg_rows_narrow=48),
                                 dict(pcg_rows_per_block=48), dict(pcg_cols_per_lane=3)])
def test_solver_parameters_are_validated(cfg1_oracle, bad):
    from paper_1912_03106_amd._abi import MgritError
    cfg = cfg1_oracle[0]
    with pytest.raises(MgritError, match="INVALID_ARGUMENT"):
        _solver(cfg, **bad)


@pytest.mark.parametrize("coarse_inverse", [0, 2])
def test_three_level_intermediate_inverse_matches_oracle(coarse_inverse):
    """3-level V-cycle with the intermediate level stepped by PCG or by its
    stored inverse (one GEMM per batched step): the oracle's history."""
    print(f"mgrit 3-level inverse {coarse_inverse}", flush=True)
    cfg = _sc_cfg()
    H, _ = build(cfg)
    n = H.levels[0].n
    U_seq = stepping.sequential(H.levels[0], np.zeros(n), cfg.n_steps)
    _, hist, _ = mgrit.solve(H, np.zeros(n), cfg.n_steps, tol=cfg.mgrit_tol, maxit=4)
    U, st = _solver(cfg, pcg_tol=1e-12, coarse_inverse=coarse_inverse).solve()
    assert st["converged"]
    for a, b in zip(st["rho"][:5], hist[:5]):
        assert abs(a - b) <= 1e-9 * hist[0], (a, b)
    assert _rel(U, U_seq) <= MGRIT_GATE


@pytest.fixture(scope="module")
def full_horizon_oracle():
    """The oracle's sequential states of the 64x512 / 16384-step workload at
    every C-point (every 16th step) and at the last F-point of every 64th
    interval, over the whole horizon (SuperLU, ~45 s on one core)."""
    cfg = config("cfg2")
    from workload import polar_mesh
    lev = stepping.Level(polar_mesh(64, 512), cfg.dt, cfg.source)
    keep = set(range(16, cfg.n_steps + 1, 16)) | set(range(15, cfg.n_steps + 1, 64 * 16))
    u = np.zeros(lev.n)
    out = {}
    for i in range(1, cfg.n_steps + 1):
        u = lev.phi(u[None], [i - 1])[0]
        if i in keep:
            out[i] = u
        if i % 4096 == 0:
            print(f"oracle 64x512: step {i}", flush=True)
    idx = np.array(sorted(out))
    return idx, np.stack([out[i] for i in idx])


@pytest.mark.parametrize("variant", ["fp64_timed", "fp32_ir"])
def test_full_size_mgrit_whole_horizon_against_oracle(full_horizon_oracle, variant):
    """The 64x512 / 16384-step / 3-level workload in the configuration
    bench.py times (F-cycles from the nested-iteration start, graph replay, no
    kernel timing), and its FP32 +
    refinement variant with the random guess: every C-point (and one F-point
    in every 64th interval) of the whole horizon against the oracle's
    sequential stepping, per time point."""
    print(f"full-size mgrit {variant}", flush=True)
    from paper_1912_03106_amd import _abi
    idx, ref = full_horizon_oracle
    timed = dict(pcg_tol_eta=3e-3, warm_start=2, residual_eta=1e-4)
    if variant == "fp64_timed":
        # F-cycles from the nested-iteration start, as timed
        cfg = config("cfg2")
        s = _solver(cfg, cycle=1, nested=1, **timed)
        assert s.params.use_graphs == 1 and s.params.profile_kernels == 0
        U, st = s.solve()
    else:
        cfg = config("cfg3")
        s = _solver(cfg, precision_coarse=_abi.FP64, **timed)
        U, st = s.solve(u_init=cfg.initial_guess(s.n0))
    s.close()
    assert st["converged"]
    assert st["rho"][-1] <= 1e-8 * st["rho"][0]
    got = U[idx]
    del U
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"{variant}: worst per-point error {err.max():.3e} at step {idx[err.argmax()]}", flush=True)
    assert err.max() <= MGRIT_GATE, (idx[err.argmax()], err.max())


def test_mgrit_degenerate_cases():
    """One coarse interval (N_t = m), a zero source (the exact solution is
    zero from the start), an empty Phi batch, and a one-level hierarchy."""
    print("mgrit degenerate", flush=True)
    from paper_1912_03106_amd import MgritError
    from workload import Source
    # N_t = m: the coarse grid has a single interval
    cfg = config("cfg1", n_steps=16, t_final=16 * config("cfg1").dt)
    H, _ = build(cfg)
    U_seq = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), 16)
    U, st = _solver(cfg, pcg_tol=1e-13).solve()
    assert st["converged"] and len(st["rho"]) <= 2
    assert _rel(U, U_seq) <= 1e-10
    # zero source: rho_0 = 0 stops at once with the zero trajectory
    cfg0 = config("cfg1", source=Source(J0=0.0))
    U0, st0 = _solver(cfg0).solve()
    assert st0["converged"] and st0["rho"] == [0.0] and not U0.any()
    # empty batch
    s = _solver(config("cfg1"))
    out = s.phi(0, np.zeros((0, s.n0)), np.zeros(0, dtype=np.int64))
    assert out.shape == (0, s.n0)
    # one level: sequential stepping works, MGRIT needs two levels
    cfg1l = config("cfg1", n_steps=64, t_final=64 * config("cfg1").dt)
    cfg1l.meshes = cfg1l.meshes[:1]
    s1 = _solver(cfg1l)
    Useq1, _ = s1.seq_solve()
    ref = stepping.sequential(H.levels[0], np.zeros(H.levels[0].n), 64)
    assert _rel(Useq1, ref) <= 1e-9
    with pytest.raises(MgritError) as e:
        s1.solve()
    assert e.value.name == "INVALID_ARGUMENT"


def test_seq_window_with_shifted_time_origin_matches_oracle():
    """GPU sequential stepping of a window whose source starts at
    t_start = 300 dt, from the oracle's state at step 300: the oracle's
    trajectory of the same steps."""
    print("seq window t_start", flush=True)
    from dataclasses import replace
    cfg = config("cfg1")
    H, _ = build(cfg)
    lev = H.levels[0]
    U = stepping.sequential(lev, np.zeros(lev.n), 364)
    wcfg = config("cfg1", n_steps=64, t_final=64 * cfg.dt,
                  source=replace(cfg.source, t_start=300 * cfg.dt))
    W, _ = _solver(wcfg, pcg_tol=1e-13).seq_solve(u0=U[300])
    err = np.linalg.norm(W - U[300:], axis=1)[1:] / np.linalg.norm(U[300:], axis=1)[1:]
    assert err.max() <= SEQ_TOL, err.max()
