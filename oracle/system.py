"""Composite system description for the oracle (test infrastructure only).

The composite Hamiltonian is a sum of local one- and two-body terms on the
graph of modes (Sec. 2.1, eq. for the Hamiltonian decomposition):

    H(t) = sum_m diag(eps_m) + sum_e g_e A_{i_e} (x) B_{j_e}
           + sum_k c_k(t) O_{m_k},

with every operator in its mode's dressed basis.  Couplings follow the
multipath form J_C n (x) n and J_L phi (x) phi (Sec. 3.1), each entered as
+g op_i (x) op_j with the sign carried by g.  Drives follow the microwave
control Hamiltonian of App. C: c(t) = E(t) cos(omega_d t + phase).

Frame (a reading: the paper does not say in which frame to step): time
stepping is done in the interaction picture of H_f = sum_m diag(eps^f_m),
where the frame energies
eps^f and the drive carriers are fixed at build from the nominal parameters
(a drive with no explicit carrier uses eps^f_1 - eps^f_0 of its mode).  At
other parameter values the generator gains diag(eps_m - eps^f_m).
"""
from __future__ import annotations

import math

import numpy as np

from .single_mode import build_mode


class OracleSystem:
    def __init__(self, desc):
        self.desc = desc
        self.modes = [build_mode(m) for m in desc["modes"]]
        self.dims = [m["d"] for m in self.modes]
        self.n_modes = len(self.dims)
        self.D = int(np.prod(self.dims))
        self.frame = []
        for md, m in zip(desc["modes"], self.modes):
            if md.get("frame_eps") is not None:
                self.frame.append(np.asarray(md["frame_eps"], dtype=np.float64)[: m["d"]])
            else:
                self.frame.append(m["eps"].copy())
        self.couplings = [dict(c) for c in desc["couplings"]]
        self.drives = []
        for dr in desc["drives"]:
            dr = dict(dr)
            if dr.get("omega_d") is None:
                f = self.frame[dr["mode"]]
                dr["omega_d"] = float(f[1] - f[0])
            self.drives.append(dr)
        self.T = float(desc["T"])
        self.N = int(desc["n_steps"])
        self.h = self.T / self.N

    # --- time grid --------------------------------------------------------
    STAGE_C = (0.0, 0.5, 0.5, 1.0)

    def stage_time(self, n, s):
        """Time of RK4 stage s (0..3) of step n: t_n + c_s h, c = (0, 1/2, 1/2, 1)."""
        return (n + self.STAGE_C[s]) * self.h

    # --- drives -------------------------------------------------------------
    def envelope(self, dr, n, t):
        """Envelope value and its derivative w.r.t. each envelope parameter."""
        env = dr["env"]
        p = np.asarray(dr["params"], dtype=np.float64)
        T = self.T
        if env == "gauss":
            sig = dr["sigma"]
            g = math.exp(-((t - 0.5 * T) ** 2) / (2.0 * sig * sig))
            return p[0] * g, np.array([g])
        if env == "gauss_basis":
            nb = len(p)
            sig = dr["sigma"]
            basis = np.array([math.exp(-((t - (j + 0.5) * T / nb) ** 2) / (2.0 * sig * sig))
                              for j in range(nb)])
            return float(basis @ p), basis
        if env == "cos_ramp":
            b = 0.5 * (1.0 - math.cos(2.0 * math.pi * t / T))
            return p[0] * b, np.array([b])
        if env == "const":
            return p[0], np.array([1.0])
        if env == "pwc":
            npc = len(p)
            piece = (n * npc) // self.N
            grad = np.zeros(npc)
            grad[piece] = 1.0
            return p[piece], grad
        raise ValueError(env)

    def drive_coeff(self, k, n, s):
        """c_k at stage s of step n, and dc_k/d(params)."""
        dr = self.drives[k]
        t = self.stage_time(n, s)
        e, de = self.envelope(dr, n, t)
        cr = math.cos(dr["omega_d"] * t + dr["phase"])
        return e * cr, de * cr

    # --- operators ----------------------------------------------------------
    def rotated(self, m, op, t):
        """Operator of mode m in the interaction picture of the frame:
        O_ab exp(i (eps^f_a - eps^f_b) t)."""
        f = self.frame[m]
        ph = np.exp(1j * (f[:, None] - f[None, :]) * t)
        return op * ph

    def op(self, m, name):
        return self.modes[m]["ops"][name]

    def delta(self, m):
        """Diagonal of H_m - H_f on mode m (zero at the nominal point)."""
        return self.modes[m]["eps"] - self.frame[m]

    # --- parameter bookkeeping -----------------------------------------------
    def n_params(self):
        return sum(len(dr["params"]) for dr in self.drives) + 3 * self.n_modes + len(self.couplings)


def build_system(desc):
    return OracleSystem(desc)
