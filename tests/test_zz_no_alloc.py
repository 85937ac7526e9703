"""The allocation-free batched Phi (phi_step_noalloc) against phi_step and
the oracle's direct-solve implicit Euler (eq. 8 as the one-step integrator of
eq. 2), through the C ABI, on two calls in a row (the second one smaller, so
that it runs on what the first left in the shared scratch array)."""

import ctypes as C

import numpy as np
import pytest

from workload import config, polar_mesh
from workload.configs import LevelSpec
from oracle.stepping import Level, sequential

pytestmark = pytest.mark.gpu

PHI_TOL = 1e-10     # relative 2-norm error per column against the direct solve


def _hip():
    """The HIP runtime libmgrit.so runs on (already loaded with it): the test,
    as the caller, allocates and copies the device arrays through it."""
    import os
    from paper_1912_03106_amd import _abi
    _abi.lib()
    hip = C.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD)
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipFree.argtypes = [C.c_void_p]
    return hip


def _dev(hip, host):
    """Device copy of a host array (hipMemcpyHostToDevice = 1)."""
    host = np.ascontiguousarray(host)
    p = C.c_void_p()
    assert hip.hipMalloc(C.byref(p), max(host.nbytes, 8)) == 0
    if host.nbytes:
        assert hip.hipMemcpy(p, host.ctypes.data_as(C.c_void_p), host.nbytes, 1) == 0
    return p


def _noalloc(s, level, u_prev, i_from):
    """phi_step_noalloc on device copies of host arrays; returns a host array."""
    hip = _hip()
    u_prev = np.ascontiguousarray(u_prev, dtype=np.float64)
    i_from = np.ascontiguousarray(i_from, dtype=np.int64)
    out = np.full_like(u_prev, np.nan)
    du, dt, do = _dev(hip, u_prev), _dev(hip, i_from), _dev(hip, out)
    try:
        rc = s._L.phi_step_noalloc(s._h, level, u_prev.shape[0], dt, du, do)
        if rc != 0:
            from paper_1912_03106_amd import MgritError
            raise MgritError(rc, s._L.mgrit_last_error(s._h).decode())
        if out.nbytes:
            assert hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), do, out.nbytes, 2) == 0
    finally:
        for p in (du, dt, do):
            hip.hipFree(p)
    return out


def _rel_cols(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("level", [0, 1])
def test_noalloc_matches_phi_step_two_calls(level, precision):
    """16x128 machine, two-level hierarchy: level 0 steps by batched PCG,
    level 1 (coarsest) by its stored inverse.  B = 200 then 37."""
    print(f"noalloc 16x128 level {level} {precision}", flush=True)
    from paper_1912_03106_amd import _abi
    from paper_1912_03106_amd.solver import Solver
    cfg = config("cfg1")
    prec = _abi.FP64 if precision == "fp64" else _abi.FP32_IR
    s = Solver(cfg, pcg_tol=1e-13, precision=prec)
    lev = Level(polar_mesh(16, 128), cfg.level_dt(level), cfg.source)
    U = sequential(lev, np.zeros(lev.n), 24)
    rng = np.random.default_rng(11 + level)
    N = cfg.level_steps(level)
    for B in (200, 37):
        # states of the workload's trajectory, scaled, plus a small perturbation
        u_prev = U[rng.integers(1, 25, size=B)] * rng.uniform(0.5, 1.5, size=(B, 1)) + \
            1e-5 * rng.standard_normal((B, lev.n))
        i_from = rng.integers(0, N - 1, size=B)
        got = _noalloc(s, level, u_prev, i_from)
        ref_gpu = s.phi(level, u_prev, i_from)
        ref = lev.phi(u_prev, i_from)
        assert np.isfinite(got).all()
        assert _rel_cols(got, ref) <= PHI_TOL
        assert _rel_cols(got, ref_gpu) <= 1e-12
    s.close()


def test_noalloc_full_size_level_at_the_limit():
    """The 64x512 level at the largest batch the scratch array holds
    (B = 64: n * 64 <= 2^21), then a smaller ragged one; B = 65 is rejected;
    the intermediate 32x256 level of the same hierarchy, two calls."""
    print("noalloc 64x512 B=64", flush=True)
    from paper_1912_03106_amd import MgritError
    from paper_1912_03106_amd.solver import Solver
    cfg = config("cfg2")
    s = Solver(cfg, pcg_tol=1e-13)
    lev = Level(polar_mesh(64, 512), cfg.dt, cfg.source)
    U = sequential(lev, np.zeros(lev.n), 24)
    rng = np.random.default_rng(5)
    for B in (64, 13):
        # states of the workload's trajectory, scaled column by column
        u_prev = U[rng.integers(4, 25, size=B)] * rng.uniform(0.2, 3.0, size=(B, 1))
        i_from = rng.integers(0, cfg.n_steps - 1, size=B)
        got = _noalloc(s, 0, u_prev, i_from)
        ref = lev.phi(u_prev, i_from)
        assert _rel_cols(got, ref) <= PHI_TOL
        assert _rel_cols(got, s.phi(0, u_prev, i_from)) <= 1e-12
    with pytest.raises(MgritError) as e:
        _noalloc(s, 0, np.zeros((65, lev.n)), np.zeros(65, dtype=np.int64))
    assert e.value.name == "INVALID_ARGUMENT"
    # the intermediate 32x256 level steps by its stored inverse (the FP64
    # matrix-core product with k split over work-groups for narrow batches)
    lev1 = Level(polar_mesh(32, 256), cfg.level_dt(1), cfg.source)
    U1 = sequential(lev1, np.zeros(lev1.n), 20)
    for B in (64, 5):
        u_prev = U1[rng.integers(2, 21, size=B)] * rng.uniform(0.5, 1.5, size=(B, 1))
        i_from = rng.integers(0, cfg.level_steps(1) - 1, size=B)
        got = _noalloc(s, 1, u_prev, i_from)
        assert _rel_cols(got, lev1.phi(u_prev, i_from)) <= PHI_TOL
        assert _rel_cols(got, s.phi(1, u_prev, i_from)) <= 1e-12
    # an empty batch is a no-op
    assert _noalloc(s, 0, np.zeros((0, lev.n)), np.zeros(0, dtype=np.int64)).shape == (0, lev.n)
    s.close()
