"""Static spectrum of the composite system (oracle; test infrastructure only).

The static Hamiltonian is the composite one of Sec. 2.1 without drives, in
the dressed single-mode bases:

    H0 = sum_m diag(eps_m) + sum_e g_e A_{i_e} (x) B_{j_e}.

Sec. 3.2 labels the composite eigenenergies by bare states (the energy
tensor): here every bare product state k gets the eigenvalue of the
eigenvector with the largest overlap |<k|v>|^2.  The static longitudinal
coupling of a pair (i, j), every other mode in its ground state, is
(Sec. 3.2, eq. for zeta_ZZI)

    zeta = E(0...0) + E(1_i 1_j) - E(1_i) - E(1_j).

Its parameter derivative follows from dE_v = <v| dH0 |v> for a
non-degenerate level v: dH0/d(E_J, E_C, E_L of mode m) is
diag(d eps_m) plus, on every coupling of m, g times the derivative of the
dressed operator of m; dH0/dg_e is A_i (x) B_j.  Parameters in the library's
order (drive parameters, which H0 does not depend on, then (E_J, E_C, E_L)
per mode, then g per coupling).
"""
from __future__ import annotations

import numpy as np

from .system import OracleSystem

DEV = ("EJ", "EC", "EL")


def _embed(sys, mats):
    """Kronecker product over the modes (mode 0 slowest); mats[m] or identity."""
    out = np.ones((1, 1), dtype=np.complex128)
    for m, d in enumerate(sys.dims):
        a = mats.get(m)
        out = np.kron(out, np.eye(d) if a is None else a)
    return out


def static_hamiltonian(sys: OracleSystem):
    H = np.zeros((sys.D, sys.D), dtype=np.complex128)
    for m, md in enumerate(sys.modes):
        H += _embed(sys, {m: np.diag(md["eps"])})
    for c in sys.couplings:
        A = sys.modes[c["i"]]["ops"][c["op_i"]]
        B = sys.modes[c["j"]]["ops"][c["op_j"]]
        H += c["g"] * _embed(sys, {c["i"]: A, c["j"]: B})
    return H


def bare_index(sys, levels):
    k = 0
    for m, d in enumerate(sys.dims):
        k = k * d + int(levels[m])
    return k


def dressed_energies(sys: OracleSystem):
    """(E_label, w, V, lab): E_label[k] is the energy of the eigenvector with
    the largest overlap with bare state k, lab[k] that eigenvector's index."""
    H = static_hamiltonian(sys)
    w, V = np.linalg.eigh(H)
    lab = np.argmax(np.abs(V) ** 2, axis=1)
    return w[lab], w, V, lab


def _pair_states(sys, i, j):
    """Bare indices of (0, 1_i 1_j, 1_i, 1_j) and their signs in zeta."""
    z = [0] * sys.n_modes
    s11, s10, s01 = list(z), list(z), list(z)
    s11[i] = s11[j] = 1
    s10[i] = 1
    s01[j] = 1
    return [bare_index(sys, z), bare_index(sys, s11), bare_index(sys, s10),
            bare_index(sys, s01)], [1.0, 1.0, -1.0, -1.0]


def static_zz(sys: OracleSystem, i, j):
    E, w, V, lab = dressed_energies(sys)
    ks, sg = _pair_states(sys, i, j)
    return float(sum(s * E[k] for k, s in zip(ks, sg)))


def static_zz_grad(sys: OracleSystem, i, j):
    """d zeta / d theta in the library's parameter order."""
    E, w, V, lab = dressed_energies(sys)
    ks, sg = _pair_states(sys, i, j)
    vs = [V[:, lab[k]] for k in ks]

    def expect(dH):
        return sum(s * float(np.real(np.vdot(v, dH @ v))) for v, s in zip(vs, sg))

    grad = [0.0] * sum(len(dr["params"]) for dr in sys.drives)
    for m, md in enumerate(sys.modes):
        for p in DEV:
            dH = _embed(sys, {m: np.diag(md["deps"][p])})
            for c in sys.couplings:
                if c["i"] == m:
                    dA = md["dops"][p][c["op_i"]]
                    B = sys.modes[c["j"]]["ops"][c["op_j"]]
                    dH = dH + c["g"] * _embed(sys, {m: dA, c["j"]: B})
                if c["j"] == m:
                    A = sys.modes[c["i"]]["ops"][c["op_i"]]
                    dB = md["dops"][p][c["op_j"]]
                    dH = dH + c["g"] * _embed(sys, {c["i"]: A, m: dB})
            grad.append(expect(dH))
    for c in sys.couplings:
        A = sys.modes[c["i"]]["ops"][c["op_i"]]
        B = sys.modes[c["j"]]["ops"][c["op_j"]]
        grad.append(expect(_embed(sys, {c["i"]: A, c["j"]: B})))
    return np.array(grad)
