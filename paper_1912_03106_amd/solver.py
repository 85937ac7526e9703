"""Python binding of the C ABI (argument marshalling only).

`Solver(cfg)` builds the mgrit_problem / mgrit_params structs from a workload
configuration and calls mgrit_setup; every computation then runs inside
libmgrit.so on the GPU:

    s = Solver(config("cfg1"))
    U, stats = s.solve()          # FAS-MGRIT, time-major [(N_t+1), n0]
    U_seq, _ = s.seq_solve()      # sequential stepping on the GPU
    u1 = s.phi(0, U[:4], [0, 1, 2, 3])   # batched Phi (eq. 2)
"""

import ctypes as C

import numpy as np

from workload import hierarchy
from workload.machine import material_arrays

from . import _abi
from ._abi import MgritError


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _check(L, h, rc):
    if rc != 0:
        msg = L.mgrit_last_error(h)
        raise MgritError(rc, msg.decode() if msg else "")


class Solver:
    """One mgrit_setup handle for a workload configuration.

    Keyword overrides set fields of mgrit_params by name (an unknown name
    raises), e.g. pcg_tol_eta=3e-3, warm_start=2, residual_eta=1e-4."""

    def __init__(self, cfg, meshes=None, stream=None, device_io=False, **overrides):
        self._L = _abi.lib()
        self.cfg = cfg
        self.meshes = meshes if meshes is not None else hierarchy(cfg)
        self.device_io = bool(device_io)
        self._keep = []
        mesh_arr = (_abi.Mesh * len(self.meshes))()
        for k, m in enumerate(self.meshes):
            arrs = dict(
                xy=np.ascontiguousarray(m.xy, dtype=np.float64),
                tri=np.ascontiguousarray(m.tri, dtype=np.int32),
                cell_mat=np.ascontiguousarray(m.cell_mat, dtype=np.int32),
                cell_phase=np.ascontiguousarray(m.cell_phase, dtype=np.int32),
                cell_sign=np.ascontiguousarray(m.cell_sign, dtype=np.int32),
                dirichlet=np.ascontiguousarray(m.dirichlet, dtype=np.uint8),
                cell_bar=np.ascontiguousarray(m.cell_bar if m.cell_bar is not None
                                              else np.full(m.n_tri, -1), dtype=np.int32),
            )
            self._keep.append(arrs)
            mesh_arr[k] = _abi.Mesh(
                m.n_r, m.n_theta, m.n_nodes, m.n_tri,
                _ptr(arrs["xy"], C.c_double), _ptr(arrs["tri"], C.c_int32),
                _ptr(arrs["cell_mat"], C.c_int32), _ptr(arrs["cell_phase"], C.c_int32),
                _ptr(arrs["cell_sign"], C.c_int32), _ptr(arrs["dirichlet"], C.c_uint8),
                _ptr(arrs["cell_bar"], C.c_int32))
        nu, sigma, iron = material_arrays()
        mats = dict(nu=np.ascontiguousarray(nu), sigma=np.ascontiguousarray(sigma),
                    iron=np.ascontiguousarray(iron, dtype=np.int32))
        self._keep.append(mats)
        src, bh = cfg.source, cfg.bh
        phys = _abi.Physics(
            len(nu), _ptr(mats["nu"], C.c_double), _ptr(mats["sigma"], C.c_double),
            _ptr(mats["iron"], C.c_int32), int(bh.nonlinear), bh.k1, bh.k2, bh.k3,
            src.J0, src.amplitude, src.freq, src.f_carrier, src.phase_offset,
            (C.c_double * 3)(*src.phases), src.carrier_code, cfg.dt, cfg.n_steps,
            src.ramp_periods, {"pwm": 0, "sine": 1}[src.signal], src.t_start)
        ct = cfg.circuit
        if ct is not None:
            phys.circuit = 1
            phys.turns_density = ct.turns_density
            phys.l_z = ct.l_z
            phys.r_phase = ct.r_phase
            phys.v0 = ct.v0
            phys.n_bars = ct.n_bars if ct.rotor else 0
            phys.ring_r = ct.ring_r
        self._mesh_arr = mesh_arr
        self._prob = _abi.Problem(len(self.meshes), mesh_arr, phys)
        par = _abi.Params()
        self._L.mgrit_default_params(C.byref(par))
        par.m = cfg.m
        par.m_coarse = cfg.m_coarse
        par.gamma = cfg.gamma
        par.precision = {"fp64": _abi.FP64, "fp32_ir": _abi.FP32_IR}[cfg.precision]
        par.tol = cfg.mgrit_tol
        par.pcg_tol = cfg.pcg_tol
        par.newton_tol = cfg.newton_tol
        par.newton_max_iter = cfg.newton_maxit
        par.newton_halvings = cfg.newton_halvings
        par.device_pointers = int(self.device_io)
        for k, v in overrides.items():
            if not hasattr(par, k):
                raise AttributeError(f"mgrit_params has no field {k}")
            setattr(par, k, v)
        self.params = par
        h = C.c_void_p()
        rc = self._L.mgrit_setup(C.byref(self._prob), C.byref(par),
                                 C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != 0:
            msg = self._L.mgrit_last_error(None)
            raise MgritError(rc, msg.decode() if msg else "")
        self._h = h

    # -- sizes -----------------------------------------------------------
    def level_info(self, level):
        """(unknowns, steps, stored operator entries) of a level."""
        n, N, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        _check(self._L, self._h, self._L.mgrit_level_info(self._h, level, C.byref(n), C.byref(N),
                                                          C.byref(nnz), None))
        return n.value, N.value, nnz.value

    def kernel_shape(self, level):
        """(rows per work-group, columns per lane, family, prefetch depth, rows
        per work-group of narrow column sets) of the level's batched PCG
        kernels as the autotuner chose them; family 1 = general sparse rows,
        2 = diagonal window; depth = rows of loads in flight per wave; the last
        is 0 when narrow sets keep the first."""
        shape = (C.c_int32 * 5)()
        _check(self._L, self._h, self._L.mgrit_level_info(self._h, level, None, None, None,
                                                          C.byref(shape)))
        return tuple(shape)

    @property
    def n0(self):
        return self.level_info(0)[0]

    # -- entry points ----------------------------------------------------
    @staticmethod
    def _check_device(t, shape):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")

    def _io(self, arr, shape, zero_ok=True):
        if arr is None:
            return None, None
        if self.device_io:
            self._check_device(arr, shape)
            return arr, C.c_void_p(arr.data_ptr())
        a = np.ascontiguousarray(arr, dtype=np.float64)
        if a.shape != shape:
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        return a, a.ctypes.data_as(C.c_void_p)

    def _out(self, out, shape):
        if self.device_io:
            if out is None:
                raise ValueError("device_io solvers need a preallocated device output")
            self._check_device(out, shape)
            return out, C.c_void_p(out.data_ptr())
        if out is None:
            out = np.empty(shape)
        return out, out.ctypes.data_as(C.c_void_p)

    def solve(self, u0=None, u_init=None, out=None, raise_on_stall=True):
        n0, N = self.n0, self.cfg.n_steps
        u0a, u0p = self._io(u0, (n0,))
        uia, uip = self._io(u_init, (N + 1, n0))
        out, outp = self._out(out, (N + 1, n0))
        st = _abi.Stats()
        rc = self._L.mgrit_solve(self._h, u0p, uip, outp, C.byref(st))
        if rc != 0 and not (rc == -7 and not raise_on_stall):
            _check(self._L, self._h, rc)
        return out, stats_dict(st)

    def joule_losses(self, out=None):
        """Joule losses P(t_i) of the last solve's iterate at every point (Sec. 3.1)."""
        N = self.cfg.n_steps
        out, outp = self._out(out, (N + 1,))
        _check(self._L, self._h, self._L.mgrit_joule_losses(self._h, outp))
        return out

    def circuit_values(self, U):
        """Stator currents [N, 3], bar voltages [N, nb] and bar currents [N, nb]
        of the steps of a level-0 trajectory U [(N+1), n0] (Sec. 3.1)."""
        ct = self.cfg.circuit
        nb = (ct.n_bars if ct.rotor else 0) if ct is not None else 0
        N, n0 = self.cfg.n_steps, self.n0
        _, up = self._io(U, (N + 1, n0))
        out = np.empty((N, 3 + 2 * nb))
        _check(self._L, self._h, self._L.mgrit_circuit_values(self._h, up, out.ctypes.data_as(C.c_void_p)))
        return out[:, :3], out[:, 3:3 + nb], out[:, 3 + nb:]

    def seq_solve(self, u0=None, out=None):
        n0, N = self.n0, self.cfg.n_steps
        u0a, u0p = self._io(u0, (n0,))
        out, outp = self._out(out, (N + 1, n0))
        st = _abi.Stats()
        _check(self._L, self._h, self._L.mgrit_seq_solve(self._h, u0p, outp, C.byref(st)))
        return out, stats_dict(st)

    def phi(self, level, u_prev, i_from):
        """Batched Phi of a level: u_prev [B, n_level], i_from [B] (host arrays)."""
        u = np.ascontiguousarray(np.atleast_2d(u_prev), dtype=np.float64)
        t = np.ascontiguousarray(np.atleast_1d(i_from), dtype=np.int64)
        if t.shape[0] != u.shape[0]:
            raise ValueError("i_from and u_prev disagree on B")
        n = self.level_info(level)[0]
        if u.shape[1] != n:
            raise ValueError(f"u_prev must have {n} columns")
        out = np.empty_like(u)
        _check(self._L, self._h, self._L.phi_step(self._h, level, u.shape[0],
                                                  t.ctypes.data_as(C.c_void_p),
                                                  u.ctypes.data_as(C.c_void_p),
                                                  out.ctypes.data_as(C.c_void_p)))
        return out

    # -- learned coarse propagator ---------------------------------------
    def coarse_n_params(self):
        return int(self._L.mgrit_coarse_n_params(self._h))

    def train_coarse(self, n_traj=64, epochs=10, batch=64, lr=2e-3, amp_spread=0.2,
                     val_fraction=0.2, seed=0, perturb=0.0):
        tp = _abi.TrainParams(n_traj, epochs, batch, lr, amp_spread, val_fraction, seed, perturb)
        ts = _abi.TrainStats()
        _check(self._L, self._h, self._L.mgrit_train_coarse(self._h, C.byref(tp), C.byref(ts)))
        return {name: getattr(ts, name) for name, _ in _abi.TrainStats._fields_}

    def set_coarse_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(self._L, self._h, self._L.mgrit_set_coarse_weights(
            self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def get_coarse_weights(self):
        w = np.empty(self.coarse_n_params(), dtype=np.float32)
        _check(self._L, self._h, self._L.mgrit_get_coarse_weights(
            self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))
        return w

    @staticmethod
    def _opt(a, B):
        if a is None:
            return None, None
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (B,)))
        return a, a.ctypes.data_as(C.c_void_p)

    def _coarse_args(self, k, u, p, amp, dphi):
        u = np.ascontiguousarray(np.atleast_2d(u), dtype=np.float64)
        p = np.ascontiguousarray(np.atleast_2d(p), dtype=np.float64)
        B = u.shape[0]
        n = self.level_info(len(self.meshes) - 1)[0]
        if u.shape != (B, n) or p.shape != (B, n):
            raise ValueError(f"u and p must be [B, {n}]")
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int64), (B,)))
        a, ap = self._opt(amp, B)
        d, dp = self._opt(dphi, B)
        keep = (u, p, k, a, d)
        return keep, B, k.ctypes.data_as(C.c_void_p), ap, dp, u.ctypes.data_as(C.c_void_p), \
            p.ctypes.data_as(C.c_void_p)

    def coarse_apply(self, k, u, p, amp=None, dphi=None):
        keep, B, kp, ap, dp, up, pp = self._coarse_args(k, u, p, amp, dphi)
        out = np.empty_like(keep[0])
        _check(self._L, self._h, self._L.mgrit_coarse_apply(self._h, B, kp, ap, dp, up, pp,
                                                            out.ctypes.data_as(C.c_void_p)))
        return out

    def coarse_gradient(self, k, u, p, y, amp=None, dphi=None):
        keep, B, kp, ap, dp, up, pp = self._coarse_args(k, u, p, amp, dphi)
        y = np.ascontiguousarray(y, dtype=np.float64)
        if y.shape != keep[0].shape:
            raise ValueError("y must match u")
        loss = C.c_double()
        g = np.empty(self.coarse_n_params(), dtype=np.float32)
        _check(self._L, self._h, self._L.mgrit_coarse_gradient(
            self._h, B, kp, ap, dp, up, pp, y.ctypes.data_as(C.c_void_p), C.byref(loss),
            g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def coarse_adam(self, grad, lr):
        g = np.ascontiguousarray(grad, dtype=np.float32)
        _check(self._L, self._h, self._L.mgrit_coarse_adam(
            self._h, g.ctypes.data_as(C.POINTER(C.c_float)), lr))

    def close(self):
        if getattr(self, "_h", None):
            self._L.mgrit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def stats_dict(st):
    k = st.n_history
    return dict(
        iterations=st.iterations, converged=bool(st.converged), rho=list(st.rho[:k]),
        phi_columns=list(st.phi_columns), pcg_sweeps=list(st.pcg_sweeps),
        newton_sweeps=list(st.newton_sweeps), time_total_s=st.time_total_s,
        time_relax_s=st.time_relax_s,
        kernel_launches=[list(st.kernel_launches[0]), list(st.kernel_launches[1])],
        kernel_columns=list(st.kernel_columns),
        kernel_time_s=[list(st.kernel_time_s[0]), list(st.kernel_time_s[1])],
        coarse_fallback=st.coarse_fallback, time_nested_s=st.time_nested_s,
        loss_change=list(st.loss_change[:k]), time_phi_s=list(st.time_phi_s),
    )
