"""Synthetic induction-machine cross-section on a structured polar mesh.

The paper's model (Sec. 3.3, a 4-pole squirrel-cage machine) and its nested
Gmsh meshes (Sec. 3.4) are not available, so a seeded, fully synthetic
stand-in with the same ingredients is generated here: an annulus with rotor
iron, conducting rotor bars, an air gap, a slotted stator carrying a
three-phase winding, and stator iron.  A = 0 on both radii (the Dirichlet
condition of Sec. 3.1).

Geometry conventions (the oracle and the HIP library both rely on them):

* nodes (i, j), i = 0..n_r, j = 0..n_theta-1, node id = i*n_theta + j,
  r_i = R_IN + i*(R_OUT-R_IN)/n_r, theta_j = 2*pi*j/n_theta;
* cell (i, j) is split along the diagonal (i,j)-(i+1,j+1) into
  T1 = [(i,j), (i+1,j), (i+1,j+1)] and T2 = [(i,j), (i+1,j+1), (i,j+1)]
  (j+1 taken modulo n_theta), both counter-clockwise; triangle id
  2*(i*n_theta+j) + {0, 1};
* a cell's material is set from its centre (R_IN+(i+1/2)dr, (j+1/2)dtheta).

Meshes with n_r, n_theta doubled are nested in the logical (i, j) sense:
coarse node (i, j) coincides with fine node (2i, 2j).
"""

from dataclasses import dataclass, field
import math

import numpy as np

R_IN = 0.02          # m, rotor inner radius (A = 0)
R_OUT = 0.10         # m, stator outer radius (A = 0)
MU0 = 4.0e-7 * math.pi

# Material ids.  Band edges are multiples of 5 mm, the radial cell size of the
# coarsest (16 x 128) mesh, so every mesh of a nested hierarchy sees the same
# radial bands.
MAT_ROTOR_IRON, MAT_BAR, MAT_AIR, MAT_SLOT, MAT_STATOR_IRON = range(5)

# name, relative permeability (linear model), conductivity S/m, iron flag
# (iron regions take the nonlinear BH law in the nonlinear model).
MATERIALS = (
    ("rotor_iron", 1000.0, 0.0, True),
    ("rotor_bar_al", 1.0, 3.5e7, False),
    ("air_gap", 1.0, 0.0, False),
    ("stator_slot", 1.0, 0.0, False),
    ("stator_iron", 1000.0, 0.0, True),
)

N_BARS = 28
N_SLOTS = 36
# 60-degree phase belts, 3 slots per pole per phase, 4 poles:
# slot group g = floor(s/3) mod 6 -> (phase, sign), phases A=0, B=1, C=2.
BELTS = ((0, +1), (2, -1), (1, +1), (0, -1), (2, +1), (1, -1))


@dataclass
class PolarMesh:
    n_r: int
    n_theta: int
    xy: np.ndarray          # [N, 2] float64, node coordinates (m)
    tri: np.ndarray         # [T, 3] int32, counter-clockwise
    cell_mat: np.ndarray    # [T] int32, material id
    cell_phase: np.ndarray  # [T] int32, -1 = no source, else 0/1/2
    cell_sign: np.ndarray   # [T] int32, winding direction (0 where no source)
    dirichlet: np.ndarray   # [N] uint8, 1 = A fixed to 0
    cell_bar: np.ndarray = None  # [T] int32, rotor bar index 0..N_BARS-1, -1 elsewhere

    @property
    def n_nodes(self) -> int:
        return self.xy.shape[0]

    @property
    def n_tri(self) -> int:
        return self.tri.shape[0]

    @property
    def n_interior(self) -> int:
        return (self.n_r - 1) * self.n_theta

    def interior_nodes(self) -> np.ndarray:
        """Node ids of the unknowns, in increasing order."""
        return np.nonzero(self.dirichlet == 0)[0].astype(np.int64)


def _cell_material(n_r: int, n_theta: int):
    dr = (R_OUT - R_IN) / n_r
    dth = 2.0 * math.pi / n_theta
    i = np.arange(n_r)[:, None]
    j = np.arange(n_theta)[None, :]
    rc = R_IN + (i + 0.5) * dr + 0.0 * j
    thc = (j + 0.5) * dth + 0.0 * i
    mat = np.full((n_r, n_theta), -1, dtype=np.int32)
    phase = np.full((n_r, n_theta), -1, dtype=np.int32)
    sign = np.zeros((n_r, n_theta), dtype=np.int32)
    eps = 1e-12
    rotor_iron = rc < 0.045 - eps
    bar_band = (rc > 0.045 - eps) & (rc < 0.055 - eps)
    air = (rc > 0.055 - eps) & (rc < 0.060 - eps)
    slot_band = (rc > 0.060 - eps) & (rc < 0.075 - eps)
    stator = rc > 0.075 - eps
    bar_pitch = 2.0 * math.pi / N_BARS
    in_bar = np.mod(thc, bar_pitch) < 0.5 * bar_pitch
    slot_pitch = 2.0 * math.pi / N_SLOTS
    in_slot = np.mod(thc, slot_pitch) < 0.5 * slot_pitch
    mat[rotor_iron] = MAT_ROTOR_IRON
    mat[bar_band & in_bar] = MAT_BAR
    mat[bar_band & ~in_bar] = MAT_ROTOR_IRON
    mat[air] = MAT_AIR
    mat[slot_band & in_slot] = MAT_SLOT
    mat[slot_band & ~in_slot] = MAT_STATOR_IRON
    mat[stator] = MAT_STATOR_IRON
    assert (mat >= 0).all()
    slot_id = np.floor(thc / slot_pitch).astype(np.int64) % N_SLOTS
    grp = (slot_id // 3) % 6
    belt_phase = np.array([b[0] for b in BELTS], dtype=np.int32)
    belt_sign = np.array([b[1] for b in BELTS], dtype=np.int32)
    coil = mat == MAT_SLOT
    phase[coil] = belt_phase[grp[coil]]
    sign[coil] = belt_sign[grp[coil]]
    bar = np.full((n_r, n_theta), -1, dtype=np.int32)
    is_bar = mat == MAT_BAR
    bar[is_bar] = (np.floor(thc / bar_pitch).astype(np.int64) % N_BARS)[is_bar]
    return mat, phase, sign, bar


def polar_mesh(n_r: int, n_theta: int) -> PolarMesh:
    """Structured triangulation of the annulus R_IN <= r <= R_OUT."""
    if n_r < 2 or n_theta < 3:
        raise ValueError("polar_mesh needs n_r >= 2 and n_theta >= 3")
    i = np.arange(n_r + 1, dtype=np.float64)
    j = np.arange(n_theta, dtype=np.float64)
    r = R_IN + i * (R_OUT - R_IN) / n_r
    th = 2.0 * math.pi * j / n_theta
    x = r[:, None] * np.cos(th)[None, :]
    y = r[:, None] * np.sin(th)[None, :]
    xy = np.stack([x.ravel(), y.ravel()], axis=1)

    ii, jj = np.meshgrid(np.arange(n_r), np.arange(n_theta), indexing="ij")
    jp = (jj + 1) % n_theta
    a = ii * n_theta + jj
    b = (ii + 1) * n_theta + jj
    c = (ii + 1) * n_theta + jp
    d = ii * n_theta + jp
    t1 = np.stack([a, b, c], axis=-1)
    t2 = np.stack([a, c, d], axis=-1)
    tri = np.stack([t1, t2], axis=2).reshape(-1, 3).astype(np.int32)

    mat, phase, sign, bar = _cell_material(n_r, n_theta)
    cell_mat = np.repeat(mat.ravel(), 2).astype(np.int32)
    cell_phase = np.repeat(phase.ravel(), 2).astype(np.int32)
    cell_sign = np.repeat(sign.ravel(), 2).astype(np.int32)
    cell_bar = np.repeat(bar.ravel(), 2).astype(np.int32)

    dirichlet = np.zeros((n_r + 1) * n_theta, dtype=np.uint8)
    dirichlet[:n_theta] = 1
    dirichlet[n_r * n_theta:] = 1
    return PolarMesh(n_r, n_theta, xy, tri, cell_mat, cell_phase, cell_sign,
                     dirichlet, cell_bar)


@dataclass
class Source:
    """Three-phase PWM current-density source (Sec. 3.2 and 3.3).

    Each coil cell carries sign * J0 * amplitude * b_phase(t), where b_p is the
    PWM signal of phase p obtained from a sine reference of frequency `freq`
    (phase angles `phases` plus a common `phase_offset`) and a carrier of
    frequency `f_carrier`.  `carrier` is "triangle" (c(0) = 1) or "sawtooth"
    (the paper's trailing-edge carrier).  `ramp_periods` > 0 multiplies the
    source by the smooth start-up factor of the nonlinear model over its first
    `ramp_periods` electric periods (0: no ramp).  `signal` "sine" drives the
    coils with the sine references themselves instead of their PWM signals
    (the smooth source of the nested-iteration start, Sec. 4.1).  `t_start`
    shifts the time origin: step i of a run samples the source at
    t_start + i*dt (a window of a longer horizon, started from a state of it).
    """
    J0: float = 1.0e7
    freq: float = 50.0
    f_carrier: float = 20.0e3
    phases: tuple = (0.0, -2.0 * math.pi / 3.0, -4.0 * math.pi / 3.0)
    carrier: str = "triangle"
    phase_offset: float = 0.0
    amplitude: float = 1.0
    ramp_periods: float = 0.0
    signal: str = "pwm"
    t_start: float = 0.0        # the source is evaluated at t_start + t (a window of the horizon)

    @property
    def carrier_code(self) -> int:
        return {"triangle": 0, "sawtooth": 1}[self.carrier]


@dataclass
class Circuit:
    """Field-circuit coupling (Sec. 3.1): the stator coils are stranded
    conductors fed by three phase voltages, the rotor bars solid conductors
    joined at both ends by resistive end rings.

    Stator: the winding function of phase s is turns_density * sign on the
    cells of phase s (turns per m^2 of slot); its current i_s is unknown and
    obeys l_z d/dt(flux integral) + r_phase i_s = v_s(t), with
    v_s(t) = v0 * amplitude * b_s(t) (times the start-up ramp when set): the
    source's PWM signals drive voltages, and Source.J0 is unused.
    Rotor (`rotor` True): bar k carries the voltage v_k and current
    i_k = G_k v_k - d/dt(integral of sigma A over bar k), G_k = sigma area_k / l_z;
    two end rings with resistance ring_r between neighbouring bars give
    i = -(1 / (2 ring_r)) L v, L the periodic path Laplacian over the bars.
    `rotor` False keeps the bars as plain conductors (v = 0).
    """
    turns_density: float = 60.0 / 8.84e-5   # 60 turns in a slot of 8.84e-5 m^2
    l_z: float = 0.1            # axial length, m
    r_phase: float = 1.5        # stator phase resistance, ohm
    v0: float = 325.0           # phase-voltage amplitude, V
    ring_r: float = 5.0e-6      # end-ring resistance between neighbouring bars, ohm
    rotor: bool = True
    n_bars: int = N_BARS


@dataclass
class BHLaw:
    """Saturating reluctivity nu(B^2) = k1*exp(k2*B^2) + k3 (A m / Wb) for iron.

    `nonlinear` False means every material uses its linear mu_r.
    """
    nonlinear: bool = False
    k1: float = 3.8
    k2: float = 2.17
    k3: float = 396.0


def material_arrays():
    """(nu_linear[5], sigma[5], iron[5]) for the material table."""
    nu = np.array([1.0 / (MU0 * m[1]) for m in MATERIALS])
    sigma = np.array([m[2] for m in MATERIALS])
    iron = np.array([1 if m[3] else 0 for m in MATERIALS], dtype=np.int32)
    return nu, sigma, iron
