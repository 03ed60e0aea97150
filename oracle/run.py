"""Build an oracle Solver from a workload dict (see workloads/__init__.py).

TEST INFRASTRUCTURE ONLY.  Units: denseness and Kn are mapped by physics.units(); the time
step is dt = cfl * dx / max|p_k| (Reading: the paper fixes dt by hand; the inputs here give
a CFL number instead).
"""
import numpy as np

from . import NG, PR_CONST, PR_ENSKOG, BC_PERIODIC, BC_EQUILIBRIUM, CHI_SET, CHI_RETFM
from . import Solver, quadrature
from . import physics


def params_of(w):
    u = physics.units(w["denseness"], w["kn"], w["kn_length"], w["n_ref"])
    p, _ = quadrature(w["q"])
    dx = w["length"] / w["nx"]
    dt = w.get("dt") or w["cfl"] * dx / np.max(np.abs(p))
    return {"b": u["b"], "mu_ref": u["mu_ref"], "dx": dx, "dt": dt, "units": u}


def rows_with_ghosts(w, field):
    """Interior values of `field` padded by the ghost states (equilibrium boundaries) or by
    periodic copies."""
    v = np.asarray(w[field], dtype=np.float64)
    idx = {"n": 0, "u": 1, "T": 2}[field]
    if w["bc"] == "periodic":
        return np.concatenate([v[-NG:], v, v[:NG]])
    return np.concatenate([np.full(NG, w["left"][idx]), v, np.full(NG, w["right"][idx])])


def solver_from_workload(w, nh=None):
    pr = params_of(w)
    s = Solver(w["nx"], w["q"], pr["dx"], pr["dt"], pr["b"], pr["mu_ref"],
               pr_mode=PR_ENSKOG if w["pr_mode"] == "enskog" else PR_CONST, pr=w["pr"],
               bc=BC_PERIODIC if w["bc"] == "periodic" else BC_EQUILIBRIUM, nh=nh,
               chi_mode=CHI_RETFM if w.get("chi", "set") == "ret" else CHI_SET,
               sigma=pr["units"]["sigma"])
    s.init_equilibrium(rows_with_ghosts(w, "n"), rows_with_ghosts(w, "u"),
                       rows_with_ghosts(w, "T"))
    s.dt = pr["dt"]
    s.units = pr["units"]
    return s
