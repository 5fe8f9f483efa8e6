"""Single-mode Hamiltonians, dressed truncation and their parameter derivatives.

Oracle (test infrastructure only).  FP64 throughout.

* Fluxonium (Sec. 3.1, eq. for the single fluxonium Hamiltonian): charging,
  inductive and Josephson terms.  Reading taken here: the external flux sits
  in the Josephson term, H = 4 E_C n^2 + E_L phi^2 / 2 - E_J cos(phi - phi_ext),
  with phi the harmonic-oscillator coordinate (for one mode this is the
  paper's form after the shift phi -> phi - phi_ext).  Represented in the
  first K harmonic-oscillator states of the charging + inductive part; the
  cosine comes from the exact matrix elements of the displacement operator
  exp(i phi) (generalised Laguerre closed form).
* Transmon (supported device type, Sec. 5.4; charge-basis form of the
  workload): H = 4 E_C (n - n_g)^2 - E_J cos(phi) in the charge basis
  |n| <= ncut, where cos(phi) hops n -> n +- 1 with amplitude 1/2.
* Dressed truncation (App. D, step 1): diagonalise, keep the lowest d levels,
  express the charge and phase operators in that eigenbasis.  Energies are
  referenced to the ground level.  Eigenvector sign: the entry of largest
  magnitude is made positive (ties within 1e-12 relative go to the lowest
  basis index).
* Derivatives (needed for device-parameter gradients, Sec. 2.1 / 2.5):
  first-order perturbation theory over the full K-state basis,
  d eps_a = v_a^T dH v_a,  d v_a = sum_{c != a} v_c (v_c^T dH v_a)/(w_a - w_c).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_genlaguerre, gammaln

SIGN_TIE_REL = 1e-12
DEGENERATE_REL = 1e-9


class DegenerateSpectrum(ValueError):
    pass


# ---------------------------------------------------------------------------
# transmon (charge basis)
# ---------------------------------------------------------------------------
def transmon_basis(EC, EJ, ng, K):
    """Charge-basis matrices: H, operators and d/d(EJ, EC, EL) of H and ops."""
    if K % 2 != 1:
        raise ValueError("transmon basis dimension must be odd (|n| <= ncut)")
    ncut = K // 2
    nvals = np.arange(-ncut, ncut + 1, dtype=np.float64)
    hop = np.eye(K, k=1) + np.eye(K, k=-1)          # 2 cos(phi) in the charge basis
    H = np.diag(4.0 * EC * (nvals - ng) ** 2) - 0.5 * EJ * hop
    nop = np.diag(nvals - ng).astype(np.complex128)
    zero = np.zeros((K, K))
    dH = {"EJ": -0.5 * hop, "EC": np.diag(4.0 * (nvals - ng) ** 2), "EL": zero}
    ops = {"n": nop}
    dops = {p: {"n": np.zeros((K, K), np.complex128)} for p in ("EJ", "EC", "EL")}
    return H, ops, dH, dops


# ---------------------------------------------------------------------------
# fluxonium (harmonic-oscillator basis)
# ---------------------------------------------------------------------------
def displacement_matrix(alpha, rows, cols):
    """<m|exp(alpha a^dag - conj(alpha) a)|n> for m < rows, n < cols (exact,
    Cahill-Glauber closed form with generalised Laguerre polynomials)."""
    x = abs(alpha) ** 2
    pref = math.exp(-0.5 * x)
    out = np.zeros((rows, cols), dtype=np.complex128)
    for m in range(rows):
        for n in range(cols):
            if m >= n:
                k = m - n
                ratio = math.exp(0.5 * (gammaln(n + 1) - gammaln(m + 1)))
                out[m, n] = ratio * alpha ** k * pref * eval_genlaguerre(n, k, x)
            else:
                k = n - m
                ratio = math.exp(0.5 * (gammaln(m + 1) - gammaln(n + 1)))
                out[m, n] = ratio * (-np.conj(alpha)) ** k * pref * eval_genlaguerre(m, k, x)
    return out


def fluxonium_basis(EC, EJ, EL, phiext, K):
    """HO-basis matrices of the fluxonium and their derivatives."""
    phi_osc = (8.0 * EC / EL) ** 0.25
    wp = math.sqrt(8.0 * EC * EL)
    k = np.arange(K, dtype=np.float64)
    a = np.diag(np.sqrt(np.arange(1, K, dtype=np.float64)), k=1)   # annihilation
    X = a + a.T                                                     # a + a^dag
    alpha = 1j * phi_osc / math.sqrt(2.0)
    Dext = displacement_matrix(alpha, K + 1, K)                     # one extra row
    D = Dext[:K, :]
    eph = np.exp(-1j * phiext)
    C = 0.5 * (eph * D + np.conj(eph) * D.conj().T)                 # cos(phi - phiext)
    if np.max(np.abs(C.imag)) > 1e-10 * max(1.0, np.max(np.abs(C.real))):
        raise AssertionError("cos(phi - phiext) not real")
    C = C.real
    H = np.diag(wp * (k + 0.5)) - EJ * C
    phi = (phi_osc / math.sqrt(2.0)) * X.astype(np.complex128)
    nop = (1j / (math.sqrt(2.0) * phi_osc)) * (a.T - a).astype(np.complex128)
    # d D / d phi_osc = P (i X / sqrt2) D P, exact in the infinite basis; the
    # product needs the row K of D, hence the extra row above.
    Xext = np.zeros((K, K + 1))
    for m in range(K):
        if m + 1 <= K:
            Xext[m, m + 1] = math.sqrt(m + 1)
        if m - 1 >= 0:
            Xext[m, m - 1] = math.sqrt(m)
    dD = (1j / math.sqrt(2.0)) * (Xext @ Dext)
    dC = 0.5 * (eph * dD + np.conj(eph) * dD.conj().T)
    dC = dC.real
    dphiosc = {"EC": phi_osc / (4.0 * EC), "EL": -phi_osc / (4.0 * EL), "EJ": 0.0}
    dwp = {"EC": wp / (2.0 * EC), "EL": wp / (2.0 * EL), "EJ": 0.0}
    dH = {}
    dops = {}
    for p in ("EJ", "EC", "EL"):
        dHp = np.diag(dwp[p] * (k + 0.5)) - EJ * dC * dphiosc[p]
        if p == "EJ":
            dHp = dHp - C
        dH[p] = dHp
        dops[p] = {"n": -nop / phi_osc * dphiosc[p], "phi": phi / phi_osc * dphiosc[p]}
    ops = {"n": nop, "phi": phi}
    return H, ops, dH, dops


# ---------------------------------------------------------------------------
# dressed truncation
# ---------------------------------------------------------------------------
def fix_signs(V):
    """Make the largest-magnitude entry of every column positive (ties within
    SIGN_TIE_REL relative go to the lowest row index)."""
    V = V.copy()
    for c in range(V.shape[1]):
        col = V[:, c]
        mag = np.abs(col)
        thr = mag.max() * (1.0 - SIGN_TIE_REL)
        idx = int(np.nonzero(mag >= thr)[0][0])
        if col[idx] < 0:
            V[:, c] = -col
    return V


def dressed_truncation(H, ops, d):
    """Eigen-decompose the basis Hamiltonian and keep the lowest d levels.

    Returns (eps[d] ground-referenced, dressed ops {name: (d,d)}, w[K], V[K,K])."""
    w, V = np.linalg.eigh(H)
    V = fix_signs(V)
    K = H.shape[0]
    scale = max(abs(w[: min(K, d + 1)]).max(), 1e-300)
    for a in range(d):
        for c in range(K):
            if c != a and abs(w[a] - w[c]) < DEGENERATE_REL * scale:
                raise DegenerateSpectrum(f"level {a} degenerate with level {c}")
    Vd = V[:, :d]
    eps = w[:d] - w[0]
    dressed = {name: Vd.T @ op @ Vd for name, op in ops.items()}
    return eps, dressed, w, V


def mode_derivatives(w, V, ops, dH, dops, d):
    """d eps (ground-referenced) and d(dressed ops) for every parameter in dH,
    from first-order perturbation theory over the full basis."""
    K = V.shape[0]
    deps = {}
    dO = {}
    for p, dHp in dH.items():
        M = V.T @ dHp @ V                        # (v_c^T dH v_a)
        dw = np.diag(M).copy()
        dV = np.zeros((K, d))
        for a in range(d):
            for c in range(K):
                if c != a:
                    dV[:, a] += V[:, c] * (M[c, a] / (w[a] - w[c]))
        deps[p] = dw[:d] - dw[0]
        Vd = V[:, :d]
        dO[p] = {}
        for name, op in ops.items():
            dO[p][name] = dV.T @ op @ Vd + Vd.T @ op @ dV + Vd.T @ dops[p][name] @ Vd
    return deps, dO


def build_mode(desc):
    """Dressed data of one mode descriptor (see scp_inputs)."""
    d = int(desc["trunc"])
    kind = desc["kind"]
    if kind == "raw":
        eps = np.asarray(desc["eps"], dtype=np.float64)
        ops = {k: np.asarray(v, dtype=np.complex128) for k, v in desc["ops"].items()}
        zero_e = np.zeros(d)
        zero_o = {k: np.zeros((d, d), np.complex128) for k in ops}
        return {"d": d, "eps": eps, "ops": ops,
                "deps": {p: zero_e for p in ("EJ", "EC", "EL")},
                "dops": {p: dict(zero_o) for p in ("EJ", "EC", "EL")}}
    K = int(desc["basis_dim"])
    if kind == "transmon":
        H, ops, dH, dops = transmon_basis(desc["EC"], desc["EJ"], desc.get("ng", 0.0), K)
    elif kind == "fluxonium":
        H, ops, dH, dops = fluxonium_basis(desc["EC"], desc["EJ"], desc["EL"],
                                           desc.get("phiext", math.pi), K)
    else:
        raise ValueError(kind)
    eps, dressed, w, V = dressed_truncation(H, ops, d)
    deps, dO = mode_derivatives(w, V, ops, dH, dops, d)
    return {"d": d, "eps": eps, "ops": dressed, "deps": deps, "dops": dO,
            "w": w, "V": V, "H": H}
