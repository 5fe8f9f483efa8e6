"""Central finite differences of the oracle loss (test only).

The frame energies and the carriers are held at their nominal values (they
are fixed at build), so each perturbed evaluation gets explicit frame
energies and explicit carrier frequencies.
"""
from __future__ import annotations

import copy

import numpy as np

from .fidelity import fidelity
from .rk4 import basis_columns, propagate
from .system import OracleSystem

DEV = ("EJ", "EC", "EL")


def frozen_desc(desc):
    """Copy of ``desc`` with the nominal frame and carriers made explicit."""
    sys0 = OracleSystem(desc)
    d = copy.deepcopy(desc)
    for m, md in enumerate(d["modes"]):
        md["frame_eps"] = sys0.frame[m].copy()
    for k, dr in enumerate(d["drives"]):
        dr["omega_d"] = sys0.drives[k]["omega_d"]
    return d


def loss(desc):
    sys = OracleSystem(desc)
    U = propagate(sys, basis_columns(sys.D, desc["columns"]))
    F, _ = fidelity(U, desc["comp_rows"], desc["comp_cols"], desc["target"])
    return 1.0 - F


def _perturbed(base, idx, delta):
    d = copy.deepcopy(base)
    i = idx
    for dr in d["drives"]:
        if i < len(dr["params"]):
            dr["params"] = list(dr["params"])
            dr["params"][i] += delta
            return d
        i -= len(dr["params"])
    for md in d["modes"]:
        if i < 3:
            md[DEV[i]] += delta
            return d
        i -= 3
    d["couplings"][i]["g"] += delta
    return d


def fd_gradient(desc, indices, step=2e-6 * np.pi, loss_fn=None):
    """Central differences dL/dtheta_i for the parameter positions ``indices``
    (loss_fn(desc) -> L; default the RK4 gate infidelity)."""
    base = frozen_desc(desc)
    f = loss if loss_fn is None else loss_fn
    out = {}
    for i in indices:
        lp = f(_perturbed(base, i, step))
        lm = f(_perturbed(base, i, -step))
        out[i] = (lp - lm) / (2.0 * step)
    return out
