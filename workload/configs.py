"""The five workload configurations and their MGRIT hierarchies.

Each configuration fixes the machine mesh, the time grid, the MGRIT
hierarchy (levels, coarsening factor m, relaxation, spatial coarsening), the
arithmetic (FP64, or FP32 inner solves with FP64 refinement), the material law
and the initial guess.  Everything here is a setting or a seeded random array;
none of it is the method's arithmetic.

Time grid: t in [0, 0.02] s (one 50 Hz period), t_i = i * dt.  Level l of an
MGRIT hierarchy uses dt_l = m**l * dt and N_l = N_t / m**l steps, or with
m_coarse > 0 the factor m between levels 0 and 1 and m_coarse below.
"""

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from .machine import Source, BHLaw, Circuit


@dataclass
class LevelSpec:
    n_r: int
    n_theta: int


@dataclass
class Config:
    name: str
    meshes: list            # LevelSpec per MGRIT level (level 0 = finest)
    n_steps: int            # N_t on level 0
    m: int                  # temporal coarsening factor
    t_final: float = 0.02
    gamma: int = 1          # number of CF relaxations after the first F (1 = FCF)
    precision: str = "fp64"  # "fp64" or "fp32_ir"
    bh: BHLaw = field(default_factory=BHLaw)
    source: Source = field(default_factory=Source)
    guess: str = "zeros"    # "zeros" or "uniform" (U(-1e-3, 1e-3), seeded)
    guess_seed: int = 0
    mgrit_tol: float = 1e-8     # relative C-point residual
    pcg_tol: float = 1e-12      # relative residual of every linear solve (FP64)
    newton_tol: float = 1e-10
    newton_maxit: int = 8
    newton_halvings: int = 6    # damping: step lengths 1, 1/2, ..., 2**-newton_halvings
    coarse: str = "implicit_euler"  # or "learned"
    m_coarse: int = 0           # coarsening factor between levels l >= 1 and l+1 (0 = m)
    circuit: Optional[Circuit] = None   # field-circuit coupling (linear model); None = current-driven coils

    @property
    def n_levels(self) -> int:
        return len(self.meshes)

    @property
    def dt(self) -> float:
        return self.t_final / self.n_steps

    def level_factors(self) -> list:
        """Temporal coarsening factor between level l and l+1, for every l."""
        mc = self.m_coarse if self.m_coarse > 0 else self.m
        return [self.m] + [mc] * max(self.n_levels - 2, 0)

    def level_steps(self, l: int) -> int:
        return self.n_steps // int(np.prod(self.level_factors()[:l], dtype=np.int64))

    def level_dt(self, l: int) -> float:
        return self.dt * int(np.prod(self.level_factors()[:l], dtype=np.int64))

    @property
    def spatial_coarsening(self) -> bool:
        return any((a.n_r, a.n_theta) != (b.n_r, b.n_theta)
                   for a, b in zip(self.meshes, self.meshes[1:]))

    def initial_guess(self, n0: int) -> np.ndarray:
        """Space-time initial guess, time-major [(N_t+1), n0].

        Row 0 is the initial value u0 = 0.  For "uniform" every later row is
        drawn from U(-1e-3, 1e-3) Wb/m with np.random.default_rng(guess_seed).
        """
        u = np.zeros((self.n_steps + 1, n0))
        if self.guess == "uniform":
            rng = np.random.default_rng(self.guess_seed)
            u[1:] = rng.uniform(-1e-3, 1e-3, size=(self.n_steps, n0))
        return u


_L16 = LevelSpec(16, 128)
_L32 = LevelSpec(32, 256)
_L64 = LevelSpec(64, 512)

_BASE = {
    # linear machine 16 x 128, 1024 steps, two-level m=16 FCF, no spatial
    # coarsening, FP64
    "cfg1": Config("cfg1", [_L16, _L16], 1024, 16),
    # same machine at 64 x 512, 16384 steps, three-level V-cycle m=16 with
    # spatial coarsening 64x512 -> 32x256 -> 16x128, batched FP64 PCG
    "cfg2": Config("cfg2", [_L64, _L32, _L16], 16384, 16),
    # cfg2 with FP32 inner PCG + FP64 refinement and a seeded random guess
    "cfg3": Config("cfg3", [_L64, _L32, _L16], 16384, 16,
                   precision="fp32_ir", guess="uniform", guess_seed=3),
    # nonlinear iron, 32768 steps over one period, three-level V m=16; the
    # source ramps in over two periods as in the nonlinear model
    "cfg4": Config("cfg4", [_L64, _L32, _L16], 32768, 16,
                   precision="fp32_ir", bh=BHLaw(nonlinear=True),
                   source=Source(ramp_periods=2.0)),
    # cfg4 with the learned coarsest-level propagator
    "cfg5": Config("cfg5", [_L64, _L32, _L16], 32768, 16,
                   precision="fp32_ir", bh=BHLaw(nonlinear=True),
                   source=Source(ramp_periods=2.0), coarse="learned"),
}

CONFIG_NAMES = tuple(_BASE)


def config(name: str, **overrides) -> Config:
    """A copy of a named configuration with optional field overrides."""
    return replace(_BASE[name], **overrides)


def hierarchy(cfg: Config):
    """Meshes of every level (generated once per distinct size)."""
    from .machine import polar_mesh
    cache = {}
    out = []
    for spec in cfg.meshes:
        key = (spec.n_r, spec.n_theta)
        if key not in cache:
            cache[key] = polar_mesh(*key)
        out.append(cache[key])
    return out
