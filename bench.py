"""Benchmark: FAS-MGRIT on the eddy-current machine workloads, one MI355X.

Headline (`value`): the linear machine on the 64 x 512 polar mesh (n = 32,256
unknowns), 16,384 implicit-Euler steps over one 50 Hz period, three-level
F-cycles (m = 16, FCF, direct spatial coarsening 64x512 -> 32x256 -> 16x128)
from the nested-iteration start (coarse problems driven by the sine
references; rho_0 is the residual of that start), batched FP64 Jacobi-PCG,
stop at a 1e-8 relative C-point residual.

One bench step = one complete MGRIT solve to the tolerance (every part of the
hot path: F/C relaxation, C-point residual, restriction, FAS right-hand side,
coarse solves, correction).  `value` is the useful throughput n0 * N_t / T of
that solve in DOF-steps/s, inputs resident on the GPU, check intervals of CG
iterations replayed from captured hipGraphs.  In the timed solve:
  - the level-0 F-relaxation solves start from the previous iterate plus the
    change of their input since it was computed;
  - the level-0 relaxation solves stop at max(1e-12 ||b||, 3e-3 ||r_0||)
    (r_0: residual of the start);
  - the C-point residual solves, which start from the current C-point values,
    stop at max(1e-12 ||b||, 1e-4 ||r_0||), i.e. at a relative accuracy of the
    residual itself;
  - the coarse levels step with stored inverses (exact implicit Euler).

Further legs of the same JSON line, run while the time budget (--budget, from
the start of the process) allows, in this order:
  - the roofline of the dominant kernel (CG pass B) from one more solve with
    HIP events around every CG pass;
  - GPU sequential stepping of the linear workload on windows spread over the
    horizon, each started from the MGRIT state at its first point (time per
    step -> full-horizon estimate; the deviation of MGRIT from the window's
    sequential states), and by the finest level's stored inverse;
  - the nonlinear machine (saturating iron, 32,768 steps, damped Newton per
    step, FP32 inner CG): time to the 1e-8 residual, and GPU sequential Newton
    stepping on windows spread over the horizon, the same way;
  - the CPU oracle timed on this host (its states also give each GPU
    solution's deviation from the oracle on its sample);
  - the FP32 + FP64-refinement variant (random initial guess);
  - the same solve with every linear solve to 1e-12 ||b|| ("plain");
  - the linear machine with the field-circuit coupling (first 4,096 steps,
    the timed solve's settings with pcg_tol 1e-14) against sequential
    stepping of the coupled model (batched CG and the stored inverse);
  - the nonlinear machine with the learned coarsest propagator (training and
    solve).
A leg that would not fit the remaining budget is listed under "skipped".
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the timed solve's pass-B and pass-A launches, from the two
# rocprofv3 --pmc runs summarised in the profile named below (each counter
# scaled by a 1 GiB copy).  Valid only for the CG kernel source (pcg.hip)
# they were taken with: reported as null once it changes.
TRAFFIC_MEASURED = {
    "sources_sha256": "f69e1baa4c52f632445b443ffea9d9d2bae6a213a22fb226e73cf9903d519227",
    "shape": [128, 1, 2, 1, 0],   # level-0 kernel shape as mgrit_level_info reports it
    "pass_b": {"bytes_per_launch": 719451950, "kernel": "k_cg_pass_b_dia<double, 1, 1>"},
    "pass_a": {"bytes_per_launch": 470357071, "kernel": "k_cg_pass_a_dia<double, 1, 1>"},
    "profile": "profiles/cg_passes_64x512_hbm_traffic.md",
}


def measured_traffic():
    """The counters' bytes per launch of passes B and A, or None once the CG
    kernel source (pcg.hip) differs from the one the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1912_03106_amd", "csrc", "pcg.hip"), "rb") as fh:
        h.update(fh.read())
    if h.hexdigest() != TRAFFIC_MEASURED["sources_sha256"]:
        return None
    return TRAFFIC_MEASURED


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pass_b_bytes(n, W, family, unit, cols, launches):
    """Algorithmic bytes of CG pass B: per unconverged column of one row, read
    p, x, r and write x, r (5 values); per launch, the level's operator
    (family 2: 8 values per row; family 1: W values + W column indices) and
    the two per-row scalings (S and diag A)."""
    matrix = n * 8 * unit if family == 2 else n * W * (unit + 4)
    return 5 * unit * n * cols + launches * (matrix + n * (unit + 8))


def pass_a_bytes(n, W, family, unit, cols, launches):
    """Algorithmic bytes of CG pass A: per unconverged column of one row, read
    r^ and the old direction and write the new one (3 values; a solve's first
    launch reads no old direction, counted as 3 all the same: about 2 % of the
    launches); per launch, the operator's diagonal and upper offsets (family
    2: 4 values per row; family 1: W values + W column indices)."""
    matrix = n * 4 * unit if family == 2 else n * W * (unit + 4)
    return 3 * unit * n * cols + launches * matrix


def pass_b_roofline(st, solver, unit):
    """Pass B over the whole timed region: algorithmic bytes / device time
    (HIP events around every launch, every level); pass A alongside."""
    T = "double" if unit == 8 else "float"
    rec = {}
    for key, pas, fbytes, tag in (("b", 1, pass_b_bytes, "b"), ("a", 0, pass_a_bytes, "a")):
        bytes_total, launches, t, cols = 0.0, 0, 0.0, 0
        names = set()
        for l in range(solver.cfg.n_levels):
            n, _, nnz = solver.level_info(l)
            rpb, cpl, fam, depth, _ = solver.kernel_shape(l)
            lau = st["kernel_launches"][pas][l]
            bytes_total += fbytes(n, nnz // n, fam, unit, st["kernel_columns"][l], lau)
            launches += lau
            cols += st["kernel_columns"][l]
            t += st["kernel_time_s"][pas][l]
            names.add(f"k_cg_pass_{tag}_dia<{T}, {cpl}, {depth}>" if fam == 2
                      else f"k_cg_pass_{tag}<{T}, {nnz // n}, {cpl}>")
        if launches == 0 or t <= 0:
            return None
        achieved = bytes_total / t / 1e9
        rec[key] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": " + ".join(sorted(names)), "launches": launches,
                    "avg_launch_us": round(1e6 * t / launches, 2),
                    "bytes_per_launch": round(bytes_total / launches),
                    "columns_per_launch": round(cols / launches, 1)}
    out = rec["b"]
    out["pass_a"] = rec["a"]
    return out


def cpu_baseline(cfg, budget_s=10.0, keep_every=64):
    """The oracle's sequential stepping (SuperLU factor + one triangular solve
    pair per step, single thread) on a prefix of the same workload.  Returns
    the JSON record and the oracle states at every keep_every-th step."""
    import numpy as np
    from workload import polar_mesh
    from oracle.stepping import Level
    spec = cfg.meshes[0]
    t0 = time.perf_counter()
    lev = Level(polar_mesh(spec.n_r, spec.n_theta), cfg.dt, cfg.source)
    t_fact = time.perf_counter() - t0
    u = np.zeros(lev.n)
    steps = 0
    kept = {}
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s and steps < cfg.n_steps:
        u = lev.phi(u[None], [steps])[0]
        steps += 1
        if steps % keep_every == 0:
            kept[steps] = u
    el = time.perf_counter() - t1
    rec = {"value": round(lev.n * steps / el, 1), "unit": "DOF-steps/s", "cores": 1,
           "kind": "oracle",
           "sample": f"sequential implicit Euler, SuperLU, first {steps} of {cfg.n_steps} steps "
                     f"on the {spec.n_r}x{spec.n_theta} mesh (factorisation {t_fact:.2f} s excluded); "
                     f"host has {os.cpu_count()} logical CPUs",
           "extrapolated_full_horizon_s": round(el / steps * cfg.n_steps + t_fact, 1)}
    return rec, kept


def oracle_deviation(kept, U):
    """max over the oracle's kept steps of ||U_gpu[i] - U_oracle[i]|| / ||U_oracle[i]||."""
    import numpy as np
    worst = 0.0
    for i, u in kept.items():
        worst = max(worst, float(np.linalg.norm(U[i] - u) / np.linalg.norm(u)))
    return worst


def timed_solve(cfg, stream, label, **kw):
    """Set up a solver, run one MGRIT solve into a device buffer, return
    (seconds, stats, solver, output tensor)."""
    import torch
    from paper_1912_03106_amd.solver import Solver
    log(f"setup {label}")
    solver = Solver(cfg, stream=stream.cuda_stream, device_io=True, **kw)
    out = torch.empty((cfg.n_steps + 1, solver.n0), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = solver.solve(out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"{label}: {len(st['rho']) - 1} iterations, {el:.2f} s")
    return el, st, solver, out


def summarize_pmc(fetch_csv, write_csv, bench_json):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the timed solve's CG
    pass-B and pass-A launches (the last `launches` dispatches of each pass in
    the run; the earlier ones belong to the set-up), each scaled by true /
    counted bytes of the 1 GiB calibration copy, and the ratio of the traffic
    to the algorithmic bytes of the same launches."""
    import csv
    with open(bench_json) as f:
        roof = json.loads(f.readline())["roofline"]
    passes = {"k_cg_pass_b": roof, "k_cg_pass_a": roof["pass_a"]}
    out = {}
    for tag, rec in passes.items():
        launches = rec["launches"]
        res = {"timed_launches": launches, "algorithmic_bytes_per_launch": rec["bytes_per_launch"]}
        for key, path, ctr in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
            pb, cp = [], []
            with open(path) as f:
                for r in csv.DictReader(f):
                    if r["Counter_Name"] != ctr:
                        continue
                    if tag in r["Kernel_Name"]:
                        pb.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
                    elif r["Kernel_Name"] == "__amd_rocclr_copyBuffer" and int(r["Grid_Size"]) >= 131072:
                        cp.append(float(r["Counter_Value"]))
            if len(pb) < launches or not cp:
                raise SystemExit(f"{path}: too few {tag} or no calibration-copy dispatches")
            pb = [v for _, v in sorted(pb)[-launches:]]
            scale = (2 ** 30 / 1024) / cp[-1]
            res[key] = {"dispatches": len(pb), "raw_kib_per_launch": sum(pb) / len(pb),
                        "calibration_copy_kib": cp[-1], "scale": scale,
                        "bytes_per_launch": 1024 * scale * sum(pb) / len(pb)}
        res["traffic_bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
        res["traffic_over_algorithmic"] = res["traffic_bytes_per_launch"] / rec["bytes_per_launch"]
        out[tag] = res
    return out


def profile_short(cfg, stream):
    """A short program for rocprofv3 --pmc: the first level-0 FCF relaxation
    and C-point residual of the timed workload (max_iter = 0), then a copy of
    2^27 doubles (1 GiB read + 1 GiB written) to calibrate the byte counters."""
    import torch
    from paper_1912_03106_amd.solver import Solver
    solver = Solver(cfg, stream=stream.cuda_stream, device_io=True, profile_kernels=1, max_iter=0,
                    **HEADLINE)
    out = torch.empty((cfg.n_steps + 1, solver.n0), dtype=torch.float64, device="cuda")
    _, st = solver.solve(out=out, raise_on_stall=False)
    torch.cuda.synchronize()
    rpb, cpl, fam, depth, _ = solver.kernel_shape(0)
    n, _, nnz = solver.level_info(0)
    lau = st["kernel_launches"][1][0]
    byts = pass_b_bytes(n, nnz // n, fam, 8, st["kernel_columns"][0], lau)
    solver.close()
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"pass_b_launches": lau, "pass_b_bytes_per_launch": round(byts / max(lau, 1)),
                      "pass_b_avg_us": round(1e6 * st["kernel_time_s"][1][0] / max(lau, 1), 2),
                      "copy_bytes": 2 * a.numel() * 8}), flush=True)


T_START = time.perf_counter()


class Budget:
    """Wall-clock budget of the whole run, counted from the start of the process."""

    def __init__(self, seconds):
        self.seconds = seconds
        self.skipped = []

    def left(self):
        return self.seconds - (time.perf_counter() - T_START)

    def fits(self, label, estimate_s):
        if self.left() >= estimate_s:
            return True
        self.skipped.append({"leg": label, "estimate_s": round(estimate_s, 1),
                             "budget_left_s": round(self.left(), 1)})
        log(f"skip {label}: needs ~{estimate_s:.0f} s, {self.left():.0f} s left")
        return False


def seq_windows(cfg_name, base, U, starts, width, stream, label, circuit=None):
    """GPU sequential stepping on windows of `width` steps starting at the
    points `starts` of the horizon of `base`, each from the MGRIT state U[i0]
    (U: the MGRIT iterate, a device tensor [(N_t+1), n0]) with the source's
    time origin moved to i0 * dt.  Returns the record: time per step (mean
    over the windows), its full-horizon estimate, and the largest relative
    deviation of the MGRIT states from the sequential ones in the windows."""
    import torch
    from dataclasses import replace
    from workload import config
    from paper_1912_03106_amd.solver import Solver
    per_step, worst, wins = [], 0.0, []
    for i0 in starts:
        wcfg = config(cfg_name, n_steps=width, t_final=width * base.dt,
                      source=replace(base.source, t_start=i0 * base.dt), circuit=circuit)
        wcfg.meshes = base.meshes[:1] * 2
        s = Solver(wcfg, stream=stream.cuda_stream, device_io=True)
        out = torch.empty((width + 1, s.n0), dtype=torch.float64, device="cuda")
        u0 = U[i0].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = s.seq_solve(u0=u0, out=out)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        s.close()
        ref = U[i0:i0 + width + 1]
        dev = float(((out[1:] - ref[1:]).norm(dim=1) / ref[1:].norm(dim=1).clamp_min(1e-300)).max())
        worst = max(worst, dev)
        per_step.append(t / width)
        wins.append({"start": i0, "steps": width, "time_s": round(t, 3),
                     "newton_per_step": round(st["newton_sweeps"][0] / width, 2) if st["newton_sweeps"][0] else None,
                     "pcg_per_step": round(st["pcg_sweeps"][0] / width, 1) if st["pcg_sweeps"][0] else None})
        log(f"{label}: window at {i0}, {width} steps, {t:.2f} s, deviation {dev:.2e}")
    ms = sum(per_step) / len(per_step)
    return {"windows": wins, "ms_per_step": round(1e3 * ms, 3),
            "time_s_full_horizon_estimate": round(ms * base.n_steps, 1),
            "mgrit_deviation_in_windows": worst}


def seq_inverse(base, U, width, stream, circuit=None):
    """GPU sequential stepping of the linear workload with the finest level's
    stored inverse (seq_kernel = 3) on the first `width` steps: build time,
    time per step (the same for every step) and its full-horizon estimate."""
    import torch
    from workload import config
    from paper_1912_03106_amd.solver import Solver
    wcfg = config("cfg2", n_steps=width, t_final=width * base.dt, circuit=circuit)
    wcfg.meshes = base.meshes[:1] * 2
    s = Solver(wcfg, stream=stream.cuda_stream, device_io=True, seq_kernel=3)
    out = torch.empty((width + 1, s.n0), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = s.seq_solve(out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.close()
    build = st["time_nested_s"]
    step = (t - build) / width
    dev = float(((out[1:] - U[1:width + 1]).norm(dim=1) / U[1:width + 1].norm(dim=1).clamp_min(1e-300)).max())
    log(f"linear sequential, stored inverse: build {build:.1f} s, {1e3 * step:.3f} ms per step")
    del out
    return {"kernel": "exact implicit-Euler steps by the stored FP64 inverse (n^2 = 8.3 GB streamed per step)",
            "steps_run": width, "inverse_build_s": round(build, 2), "ms_per_step": round(1e3 * step, 3),
            "time_s_full_horizon_estimate": round(build + step * base.n_steps, 1),
            "mgrit_deviation": dev}


CIRCUIT_STEPS = 4096      # the field-circuit leg: the first quarter of the 16384-step horizon
# coupled solves with early stops: the ||b||-relative floor of the stop
# (b = (M/dt) a is dominated by the bars' sigma/dt rows) is set 100x tighter
# than the uncoupled model's, or MGRIT levels off near 1e-8 of rho_0
CIRCUIT_PCG_TOL = 1e-14


def circuit_leg(stream, seq_width=32):
    """The linear workload with the field-circuit coupling (voltage-driven
    stranded stator coils, rotor bars joined by resistive end rings) on the
    first CIRCUIT_STEPS steps: MGRIT with the timed solve's settings and
    pcg_tol = CIRCUIT_PCG_TOL, the set-up
    (coupling solves Z = A^-1 B^T per level), the peak currents, and the
    deviation from GPU sequential stepping of the coupled model on four
    windows spread over the horizon."""
    import torch
    from workload import config, Circuit
    from paper_1912_03106_amd.solver import Solver
    full = config("cfg2")
    cfg = config("cfg2", circuit=Circuit(), n_steps=CIRCUIT_STEPS, t_final=CIRCUIT_STEPS * full.dt)
    log("field-circuit: setup")
    t_set = time.perf_counter()
    s = Solver(cfg, stream=stream.cuda_stream, device_io=True, pcg_tol=CIRCUIT_PCG_TOL, **HEADLINE)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_set
    out = torch.empty((cfg.n_steps + 1, s.n0), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = s.solve(out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    i1, v2, i2 = s.circuit_values(out)
    s.close()
    rho = st["rho"]
    log(f"field-circuit: {len(rho) - 1} iterations, {t:.2f} s")
    N = cfg.n_steps
    rec = {"workload": f"the linear 64x512 workload, first {N} of 16384 steps, with voltage-driven "
                       "stranded stator coils (325 V PWM, 1.5 ohm) and 28 rotor bars joined by resistive "
                       "end rings; the timed solve's settings (3-level F-cycles from the nested start, "
                       "level-0 relaxation solves stopped at 3e-3 of their start residual, C-point "
                       "residual solves at 1e-4) with pcg_tol 1e-14; coupled solves start from the "
                       "previous iterate less Z times the stored circuit unknowns, and the circuit "
                       "unknowns come from the exact circuit rows of each step (the solve's residual "
                       "folded in)",
           "time_to_solution_s": round(t, 3), "iterations": len(rho) - 1, "rho_rel_final": rho[-1] / rho[0],
           "setup_s": round(setup_s, 2), "dof_steps_per_s": round(32256 * N / t, 1),
           "stator_current_peak_a": round(float(abs(i1).max()), 2),
           "bar_current_peak_a": round(float(abs(i2).max()), 1)}
    rec["gpu_sequential"] = seq_windows("cfg2", cfg, out, [N // 8, 3 * N // 8, 5 * N // 8, 7 * N // 8],
                                        seq_width, stream, "field-circuit sequential", circuit=cfg.circuit)
    rec["gpu_sequential"]["kernel"] = "the batched step and its circuit elimination on one column (1e-12)"
    # the same stepping with the level's stored inverse (exact steps) and the
    # circuit elimination after each
    inv = seq_inverse(cfg, out, 1024, stream, circuit=cfg.circuit)
    inv["kernel"] = ("exact implicit-Euler steps by the stored FP64 inverse, then the circuit "
                     "elimination")
    rec["gpu_sequential"]["stored_inverse"] = inv
    ref = min(rec["gpu_sequential"]["time_s_full_horizon_estimate"], inv["time_s_full_horizon_estimate"])
    rec["gpu_sequential"]["fastest_full_horizon_s"] = ref
    rec["speedup_vs_gpu_sequential"] = round(ref / t, 3)
    del out
    return rec


NL_ETA = 1e-3            # nonlinear level-0 relaxation: stop at eta times the start residual
# the nonlinear legs' solver settings: V-cycles from the nested-iteration
# start (31 instead of 36 iterations on 8192 steps, 10 % faster; F-cycles
# were slower there)
NL_SETTINGS = dict(pcg_tol_eta=NL_ETA, nested=1)
NL_ESTIMATE_S = 190.0    # nonlinear 32768-step leg: MGRIT, set-up and the sequential windows


def nonlinear_leg(N, stream, budget=None, learned=False, profile=False, seq_width=32, ie=True):
    """The saturating-iron workload (64x512, dt = 0.02/32768, start-up ramp,
    damped Newton, FP32 inner CG + FP64 Newton residual, 3-level V-cycle) on
    its first N steps: MGRIT with implicit Euler on the coarse levels, GPU
    sequential Newton stepping on four windows spread over the horizon, and
    optionally the learned coarsest propagator."""
    from workload import config
    full = config("cfg4")
    cfg = config("cfg4", n_steps=N, t_final=N * full.dt)
    rec = {"workload": f"nonlinear eddy-current machine 64x512 (Brauer iron, ramp over 2 periods), "
                       f"{N} of 32768 steps (dt = {full.dt:.3e} s), 3-level V-cycles from the "
                       f"nested-iteration start, m=16, with spatial "
                       f"coarsening, damped Newton, FP32 inner CG + FP64 Newton residual, level-0 "
                       f"relaxation stopped at {NL_ETA:g} of the start residual"}
    t = None
    if ie:
        t = _nonlinear_ie(rec, cfg, N, stream, budget, profile, seq_width)
    if learned and (budget is None or budget.fits("nonlinear learned", 2.2 * (t or 180.0) + 60.0)):
        _nonlinear_learned(rec, cfg, N, stream)
    return rec


def _nonlinear_ie(rec, cfg, N, stream, budget, profile, seq_width):
    import torch
    from paper_1912_03106_amd.solver import Solver
    log("nonlinear: setup")
    t_set = time.perf_counter()
    s = Solver(cfg, stream=stream.cuda_stream, device_io=True, profile_kernels=int(profile),
               **NL_SETTINGS)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_set
    out = torch.empty((N + 1, s.n0), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = s.solve(out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    rho = st["rho"]
    rec["implicit_euler"] = {"time_to_solution_s": round(t, 2), "iterations": len(rho) - 1,
                             "rho_rel_final": rho[-1] / rho[0], "setup_s": round(setup_s, 2),
                             "newton_sweeps": st["newton_sweeps"][:3], "pcg_sweeps": st["pcg_sweeps"][:3],
                             "dof_steps_per_s": round(s.n0 * N / t, 1)}
    if profile:
        rec["implicit_euler"]["time_phi_s"] = [round(x, 2) for x in st["time_phi_s"][:3]]
    log(f"nonlinear: {len(rho) - 1} iterations, {t:.1f} s")
    s.close()
    starts = [N // 8, 3 * N // 8, 5 * N // 8, 7 * N // 8]
    if budget is None or budget.fits("nonlinear sequential windows", 15.0):
        rec["gpu_sequential"] = seq_windows("cfg4", cfg, out, starts, seq_width, stream,
                                            "nonlinear sequential")
        rec["gpu_sequential"]["kernel"] = "damped Newton on one column, same batched kernels, strict tolerances"
        rec["implicit_euler"]["speedup_vs_gpu_sequential"] = round(
            rec["gpu_sequential"]["time_s_full_horizon_estimate"] / t, 3)
    del out
    return t


def _nonlinear_learned(rec, cfg, N, stream):
    """The same solve with the learned coarsest propagator (implicit Euler plus
    the network correction), trained on the GPU first."""
    import torch
    from paper_1912_03106_amd.solver import Solver
    log("nonlinear learned coarse propagator: training")
    s = Solver(cfg, stream=stream.cuda_stream, device_io=True, coarse_model=1, **NL_SETTINGS)
    ts = s.train_coarse(n_traj=128, epochs=8, batch=64, lr=2e-3, seed=5, perturb=0.3)
    log(f"nonlinear learned: trained ({ts['time_data_s']:.0f} s data, {ts['time_train_s']:.0f} s Adam)")
    out = torch.empty((N + 1, s.n0), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, lst = s.solve(out=out)
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    rec["learned"] = {"time_to_solution_s": round(tl, 2), "iterations": len(lst["rho"]) - 1,
                      "coarse_fallback": lst["coarse_fallback"],
                      "training": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in ts.items()}}
    log(f"nonlinear learned: {len(lst['rho']) - 1} iterations, {tl:.1f} s")
    s.close()
    del out


HEADLINE_ETA = 3e-3      # level-0 relaxation: stop at max(pcg_tol ||b||, eta ||r_0||)
FP32_ETA = 3e-3
RESIDUAL_ETA = 1e-4      # C-point residual solves: relative accuracy of the residual
# the timed solver settings: F-cycles from the nested-iteration start (the
# coarse problems driven by the sine references, Sec. 4.1), F-relaxation
# solves started from the previous iterate plus the change of their input
# (warm_start = 2)
HEADLINE = dict(pcg_tol_eta=HEADLINE_ETA, warm_start=2, residual_eta=RESIDUAL_ETA, cycle=1, nested=1)


def pinned(shape):
    """Solver settings that fix the level-0 batched-CG kernel shape (as
    mgrit_level_info reports it) instead of autotuning it."""
    rpb, cpl, fam, depth, narrow = shape
    return dict(pcg_kernel=fam, pcg_rows_per_block=rpb, pcg_cols_per_lane=cpl, pcg_prefetch=depth,
                pcg_rows_narrow=narrow if narrow > 0 else -1)


def profiled_settings(args):
    """The profiled (roofline) solve: the headline settings, with the kernel
    shape the HBM counters were taken with, so that the measured traffic
    belongs to the kernel whose time is measured."""
    kw = dict(HEADLINE)
    if TRAFFIC_MEASURED["shape"] and not args.pin_shape:
        kw.update(pinned(TRAFFIC_MEASURED["shape"]))
    return kw


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--budget", type=float, default=555.0,
                    help="seconds for the whole run (from the start of the process); legs after "
                         "the headline that would not fit are skipped and listed")
    ap.add_argument("--seq-width", type=int, default=512,
                    help="steps per window of the linear GPU sequential baseline (4 windows)")
    ap.add_argument("--no-seq", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the plain-tolerance and FP32 + refinement solves")
    ap.add_argument("--no-nonlinear", action="store_true", help="skip the nonlinear legs")
    ap.add_argument("--nonlinear", type=int, default=0, metavar="N",
                    help="instead: only the saturating-iron workload on its first N steps (N "
                         "divisible by 256), with the learned coarse propagator too")
    ap.add_argument("--no-circuit", action="store_true", help="skip the field-circuit leg")
    ap.add_argument("--circuit", action="store_true",
                    help="instead: only the field-circuit leg (the timed linear workload with "
                         "voltage-driven coils and the rotor cage)")
    ap.add_argument("--nl-skip-learned", action="store_true",
                    help="with --nonlinear: skip the learned coarse propagator run")
    ap.add_argument("--nl-profile", action="store_true",
                    help="with --nonlinear: wall time per level (stream drained around every Phi)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed solve, copy 2^27 doubles (1 GiB read, 1 GiB written) so that "
                         "rocprofv3 byte counters can be calibrated on a kernel of known traffic")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="print the per-launch HBM traffic of CG pass B from two rocprofv3 --pmc "
                         "counter_collection.csv files (FETCH_SIZE, WRITE_SIZE), calibrated by the copy; "
                         "the last `launches` pass-B dispatches (from the bench line of the same run) "
                         "are the timed solve's")
    ap.add_argument("--pin-shape", metavar="RPB,CPL,DEPTH,NARROW",
                    help="pin the level-0 batched-CG kernel shape (rows per work-group, columns per "
                         "lane, prefetch depth, narrow-set rows per work-group, 0 = none) instead of "
                         "autotuning it: hardware-counter runs distort the autotuner's timings")
    ap.add_argument("--profile-short", action="store_true",
                    help="for hardware-counter runs: one level-0 relaxation and C-point residual "
                         "of the 64x512 workload, then a 1 GiB device copy of known size")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc)))
        return
    if args.pin_shape:
        rpb, cpl, depth, narrow = (int(v) for v in args.pin_shape.split(","))
        HEADLINE.update(pinned((rpb, cpl, 2, depth, narrow)))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the time-parallel "
              "decomposition over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from workload import config
    from paper_1912_03106_amd import _abi
    from paper_1912_03106_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    budget = Budget(args.budget)
    cfg = config("cfg2")
    if args.profile_short:
        profile_short(cfg, stream)
        return
    if args.nonlinear:
        print(json.dumps(nonlinear_leg(args.nonlinear, stream, learned=not args.nl_skip_learned,
                                       profile=args.nl_profile)), flush=True)
        return
    if args.circuit:
        print(json.dumps(circuit_leg(stream)), flush=True)
        return

    # headline: timed solves, check intervals of CG iterations replayed from
    # captured hipGraphs, no per-kernel timing
    log("setup cfg2 (timed)")
    t_setup = time.perf_counter()
    solver = Solver(cfg, stream=stream.cuda_stream, device_io=True, **HEADLINE)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    n0 = solver.n0
    out = torch.empty((cfg.n_steps + 1, n0), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for w in range(args.warmup):
        solver.solve(out=out)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        _, st = solver.solve(out=out)
        stats.append(st)
        log(f"solve {k + 1}/{args.steps}: {len(st['rho']) - 1} iterations, {st['time_total_s']:.2f} s")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = stats[-1]
    per = el / args.steps
    value = n0 * cfg.n_steps / per
    rho = st["rho"]
    n_t = cfg.level_steps(1)                     # intervals = C-point residual columns per iteration
    frelax_cols = st["phi_columns"][0] - len(rho) * n_t
    shapes = [dict(zip(("rows_per_block", "cols_per_lane", "family", "prefetch_rows", "rows_per_block_narrow"),
                       solver.kernel_shape(l)))
              for l in range(cfg.n_levels)]
    solver.close()

    # the roofline of the dominant kernel: one more solve of the same
    # workload with HIP events around every CG pass (eager launches)
    roof, pst, t_prof = None, None, None
    if budget.fits("profiled solve", 1.3 * per + 5.0):
        log("profiled solve (HIP events around every CG pass)")
        psolver = Solver(cfg, stream=stream.cuda_stream, device_io=True, profile_kernels=1,
                         **profiled_settings(args))
        pout = torch.empty_like(out)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        _, pst = psolver.solve(out=pout)
        torch.cuda.synchronize()
        t_prof = time.perf_counter() - tp0
        roof = pass_b_roofline(pst, psolver, 8)
        if roof is not None:
            tm = measured_traffic()
            shape0 = list(psolver.kernel_shape(0))
            roof["shape"] = shape0
            if tm is not None and shape0 != tm["shape"]:
                roof["traffic_note"] = (f"counters were taken with level-0 kernel shape {tm['shape']}; "
                                        f"this run's autotuner chose {shape0}")
                tm = None
            if tm is not None:
                for rec, key in ((roof, "pass_b"), (roof["pass_a"], "pass_a")):
                    rec["traffic"] = tm[key]["bytes_per_launch"]
                    rec["traffic_over_algorithmic"] = round(rec["traffic"] / rec["bytes_per_launch"], 3)
                    rec["traffic_kernel"] = tm[key]["kernel"]
                roof["traffic_profile"] = tm["profile"]
        psolver.close()
        del pout
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # linear GPU sequential stepping on windows of the horizon
    seq = None
    if not args.no_seq and budget.fits("linear sequential windows", 4 * args.seq_width * 0.0045 + 8.0):
        N = cfg.n_steps
        seq = seq_windows("cfg2", cfg, out, [0, N // 4, N // 2, 3 * N // 4], args.seq_width, stream,
                          "linear sequential")
        seq["kernel"] = "cooperative multi-work-group Jacobi-PCG stepper (warm start u_{i-1}, 1e-12)"
    # the same stepping with the level's stored inverse (exact steps, one
    # stream of the 8.3 GB inverse per step; cost independent of the state)
    if not args.no_seq and budget.fits("linear sequential, stored inverse", 45.0):
        seq_inv = seq_inverse(cfg, out, args.seq_width * 2, stream)
        if seq is None:
            seq = {}
        seq["stored_inverse"] = seq_inv
    # the largest workload: the nonlinear machine over its whole horizon
    nl = None
    if not args.no_nonlinear and budget.fits("nonlinear 32768 steps", NL_ESTIMATE_S):
        nl = nonlinear_leg(config("cfg4").n_steps, stream, budget=budget)

    U_head = out.cpu().numpy()
    del out

    cpu = None
    if not args.no_cpu and budget.fits("CPU oracle sample", 15.0):
        log("CPU oracle sample")
        cpu, kept = cpu_baseline(cfg)
        cpu["gpu_deviation_on_sample"] = {"timed_solve": oracle_deviation(kept, U_head)}

    variants = {}
    if not args.no_variants and budget.fits("FP32 + refinement", 0.9 * per + 8.0):
        cfg3 = config("cfg3")
        guess = torch.from_numpy(cfg3.initial_guess(n0)).to("cuda")
        log("setup cfg3 FP32 + refinement")
        vs = Solver(cfg3, stream=stream.cuda_stream, device_io=True, pcg_tol_eta=FP32_ETA,
                    warm_start=2, residual_eta=RESIDUAL_ETA, precision_coarse=_abi.FP64)
        vout = torch.empty_like(guess)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, vst = vs.solve(u_init=guess, out=vout)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        log(f"FP32 + refinement: {len(vst['rho']) - 1} iterations, {t:.2f} s")
        variants["fp32_ir"] = {"time_to_solution_s": round(t, 3), "iterations": len(vst["rho"]) - 1,
                               "pcg_sweeps": vst["pcg_sweeps"][:cfg.n_levels],
                               "guess": "U(-1e-3, 1e-3), seed 3",
                               "level0_stop": f"max(1e-12 ||b||, {FP32_ETA:g} ||r_0||), F-relaxation "
                                              "from the previous iterate plus its input's change, "
                                              f"C-point residual to {RESIDUAL_ETA:g} relative",
                               "coarse_levels": "stored inverses (FP64)"}
        U = vout.cpu().numpy()
        variants["fp32_ir"]["rel_diff_vs_timed_solve"] = float(np.linalg.norm(U - U_head) / np.linalg.norm(U_head))
        if cpu is not None:
            cpu["gpu_deviation_on_sample"]["fp32_ir"] = oracle_deviation(kept, U)
        vs.close()
        del vout, guess, U

    if not args.no_variants and budget.fits("plain FP64", 4.5 * per + 8.0):
        t, vst, vs, vout = timed_solve(cfg, stream, "plain FP64 (every solve to 1e-12)")
        variants["plain_fp64"] = {"time_to_solution_s": round(t, 3), "iterations": len(vst["rho"]) - 1,
                                  "pcg_sweeps": vst["pcg_sweeps"][:cfg.n_levels]}
        U = vout.cpu().numpy()
        variants["plain_fp64"]["rel_diff_vs_timed_solve"] = float(np.linalg.norm(U - U_head) / np.linalg.norm(U_head))
        if cpu is not None:
            cpu["gpu_deviation_on_sample"]["plain_fp64"] = oracle_deviation(kept, U)
        vs.close()
        del vout, U
    circ = None
    if not args.no_circuit and budget.fits("field-circuit", 55.0):
        from paper_1912_03106_amd._abi import MgritError
        try:
            circ = circuit_leg(stream)
        except MgritError as e:
            # a solver error of this leg goes into the line; it does not end the run
            log(f"field-circuit leg failed: {e}")
            circ = {"error": str(e)}
    if nl is not None and budget.fits("nonlinear learned", 2.2 * nl["implicit_euler"]["time_to_solution_s"] + 60.0):
        nl["learned"] = nonlinear_leg(config("cfg5").n_steps, stream, budget=budget, learned=True,
                                      ie=False).get("learned")

    line = {
        "metric": "MGRIT time to 1e-8 rel. resid vs GPU seq. stepping; F-relax DOF-steps/s, GB/s",
        "value": round(value, 1), "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * per, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "linear eddy-current machine, 64x512 polar P1 mesh (n=32256), "
                               "16384 implicit-Euler steps over 0.02 s, PWM 20 kHz; 3-level F-cycles "
                               "(m=16, FCF) from the nested-iteration start (coarse problems driven by "
                               "the sine references; rho_0 is the residual of that start), spatial "
                               "coarsening 64x512/32x256/16x128; FP64 Jacobi-PCG; "
                               f"level-0 relaxation solves stop at max(1e-12 ||b||, {HEADLINE_ETA:g} "
                               "||r_0||), F-relaxation solves start from the previous iterate plus "
                               "the change of their input; C-point residual solves at max(1e-12 "
                               f"||b||, {RESIDUAL_ETA:g} ||r_0||) from the current C-point values; "
                               "coarse levels by stored inverses (FP64 GEMM on 32x256, inverse "
                               "apply on 16x128)",
                   "n_dof": n0, "n_steps": cfg.n_steps, "levels": cfg.n_levels, "m": cfg.m},
        "roofline": roof,
        "cpu_baseline": cpu,
        "mgrit": {"time_to_solution_s": round(per, 3), "iterations": len(rho) - 1,
                  "rho_rel_final": rho[-1] / rho[0] if rho and rho[0] else None,
                  "frelax_dof_steps_per_s": round(n0 * frelax_cols / st["time_relax_s"], 1)
                  if st["time_relax_s"] > 0 else None,
                  "level0_phi": frelax_cols, "pcg_sweeps": st["pcg_sweeps"][:cfg.n_levels],
                  "setup_s": round(setup_s, 2), "nested_start_s": round(st["time_nested_s"], 3),
                  "autotuned_kernels": shapes},
        "nonlinear": nl,
        "variants": variants or None,
        "field_circuit": circ,
        "gpu_sequential": seq,
        "skipped": budget.skipped or None,
        "wall_s": round(time.perf_counter() - T_START, 1),
    }
    if pst is not None:
        line["mgrit"]["profiled_solve"] = {
            "time_s": round(t_prof, 3), "iterations": len(pst["rho"]) - 1,
            "pass_a_time_s": [round(x, 3) for x in pst["kernel_time_s"][0][:cfg.n_levels]],
            "pass_b_time_s": [round(x, 3) for x in pst["kernel_time_s"][1][:cfg.n_levels]]}
    if seq:
        # the fastest GPU sequential method is the reference
        cands = [x["time_s_full_horizon_estimate"] for x in (seq, seq.get("stored_inverse") or {})
                 if "time_s_full_horizon_estimate" in x]
        ref = min(cands)
        seq["fastest_full_horizon_s"] = ref
        line["mgrit"]["speedup_vs_gpu_sequential"] = round(ref / per, 3)
        for v in variants.values():
            v["speedup_vs_gpu_sequential"] = round(ref / v["time_to_solution_s"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
