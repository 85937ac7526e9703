"""Build the oracle's MGRIT hierarchy for a workload configuration.

Level l uses the mesh of the configuration's l-th entry and the step
dt_l = m**l * dt (coarse propagators are re-discretisations with the coarse
step, Sec. 2.1).  Spatial transfers between differing meshes are P_s and
R_s = D^{-1} P_s^T from `transfer.py`; equal meshes use none.  With a
field-circuit configuration every level is the coupled model of
`circuit.py`; MGRIT's state stays the vector potential.
"""

from workload import hierarchy as mesh_hierarchy

from .fe import MachineFE
from .mgrit import Hierarchy
from .stepping import Level
from .circuit import CircuitLevel
from . import transfer


def build(cfg, restriction="normalized"):
    meshes = mesh_hierarchy(cfg)
    fes = {}
    levels = []
    for l, mesh in enumerate(meshes):
        key = (mesh.n_r, mesh.n_theta)
        if key not in fes:
            fes[key] = MachineFE(mesh)
        if cfg.circuit is not None:
            if cfg.bh.nonlinear:
                raise NotImplementedError("the field-circuit model is linear here")
            levels.append(CircuitLevel(mesh, cfg.level_dt(l), cfg.source, cfg.circuit, fe=fes[key]))
            continue
        levels.append(Level(mesh, cfg.level_dt(l), cfg.source, cfg.bh, fe=fes[key],
                            newton_tol=cfg.newton_tol, newton_maxit=cfg.newton_maxit,
                            newton_halvings=cfg.newton_halvings))
    R, P = [], []
    for fine, coarse in zip(meshes, meshes[1:]):
        if (fine.n_r, fine.n_theta) == (coarse.n_r, coarse.n_theta):
            R.append(None)
            P.append(None)
        else:
            Ps = transfer.prolongation(fine, coarse)
            P.append(Ps)
            R.append(transfer.restriction(Ps, restriction)
                     if restriction != "injection" else transfer.injection(fine, coarse))
    return Hierarchy(levels, cfg.level_factors(), R=R, P=P, gamma=cfg.gamma), meshes
