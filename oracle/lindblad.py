"""Open-system propagation: the vectorised Lindblad master equation
(oracle; test infrastructure only).

The paper carries its propagation and back-propagation over to open systems:
a density matrix evolves under a superoperator obtained from the vectorised
Lindblad master equation (App. D, closing remark on the average fidelity;
the LindbladObj component of Sec. 2).  It fixes neither the jump operators nor
their rates.  Readings:
  - two channels per mode m, in the mode's dressed basis: energy relaxation
    L = sqrt(gamma1_m) a_m with the ladder a = sum_k sqrt(k) |k-1><k|, and
    pure dephasing L = sqrt(2 gammaphi_m) n_m with n = diag(0, 1, .., d-1),
    so that the 0-1 coherence of an idle mode decays as exp(-gammaphi t) and
    its excited population as exp(-gamma1 t);
  - the equation is stepped in the interaction picture of the closed system's
    frame H_f (system.py): rho_I = exp(i H_f t) rho exp(-i H_f t) obeys
        d rho_I/dt = -i [V(t), rho_I]
                     + sum_j ( L_j(t) rho_I L_j(t)^dag
                               - 1/2 {L_j(t)^dag L_j(t), rho_I} ),
    V(t) the closed system's interaction-picture generator and
    L_j(t) = exp(i H_f t) L_j exp(-i H_f t);
  - classical RK4 on the closed system's grid (Sec. 2.3 fixed steps), applied
    to this linear equation for rho.

Average gate fidelity (App. D, eq. for the average fidelity, after Nielsen):
F = (sum_j tr(U U_j^dag U^dag E(U_j)) + d^2) / (d^2 (d + 1)) with U the target
and U_j a basis of unitary operators normalised to tr(U_j^dag U_k) = d delta_jk
(reading: the printed "orthonormal" basis needs this normalisation for F = 1
at a perfect gate).  The sum is d times the trace of the superoperator
U^dag E(.) U, which in the matrix-unit basis E_ab = |a><b| of the input states
gives
    F = (Re sum_ab <u_a| E(E_ab) |u_b> + d) / (d (d + 1)),
u_a the target's column a placed on the computational rows (the real part:
the sum is real for any Hermiticity-preserving map).  For a unitary channel W
this is (|tr(U^dag W)|^2 + d) / (d (d + 1)).

Gradient: discrete adjoint of the RK4 steps, as for the closed system
(adjoint.py), with A_s = L(t_s) and its adjoint
    L^dag(X) = i [V, X] + sum_j ( L_j^dag X L_j - 1/2 {L_j^dag L_j, X} ),
convention dLoss = 2 Re <lambda, d rho>, <A, B> = tr(A^dag B).
Parameters: the drive parameters (drive order), the coupling strengths, then
(gamma1_m, gammaphi_m) of every mode.  The device parameters (E_J, E_C, E_L)
are not differentiated on this path.

Everything here is dense D x D matrices built with Kronecker products: slow
and plain on purpose.
"""
from __future__ import annotations

import numpy as np


def rates(desc):
    """Per-mode (gamma1, gammaphi) in 1/ns; absent keys mean zero."""
    g1 = np.array([float(m.get("gamma1", 0.0)) for m in desc["modes"]])
    gp = np.array([float(m.get("gammaphi", 0.0)) for m in desc["modes"]])
    return g1, gp


def embed(op, m, dims):
    """I (x) .. op on mode m .. (x) I as a dense D x D matrix (mode 0 slowest)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for k, d in enumerate(dims):
        out = np.kron(out, op if k == m else np.eye(d, dtype=np.complex128))
    return out


def ladder(d):
    a = np.zeros((d, d), dtype=np.complex128)
    for k in range(1, d):
        a[k - 1, k] = np.sqrt(k)
    return a


def number(d):
    return np.diag(np.arange(d, dtype=np.float64)).astype(np.complex128)


def generator(sys, n, s):
    """Dense interaction-picture Hamiltonian V(t) at RK4 stage s of step n and
    the dense operators dV/dp of the drive parameters and coupling strengths."""
    t = sys.stage_time(n, s)
    dims = sys.dims
    V = np.zeros((sys.D, sys.D), dtype=np.complex128)
    for m in range(sys.n_modes):
        V += embed(np.diag(sys.delta(m)).astype(np.complex128), m, dims)
    dpar = []
    for k, dr in enumerate(sys.drives):
        c, dc = sys.drive_coeff(k, n, s)
        O = embed(sys.rotated(dr["mode"], sys.op(dr["mode"], dr["op"]), t), dr["mode"], dims)
        V += c * O
        for v in dc:
            dpar.append(v * O)
    dcoup = []
    for cp in sys.couplings:
        A = embed(sys.rotated(cp["i"], sys.op(cp["i"], cp["op_i"]), t), cp["i"], dims)
        B = embed(sys.rotated(cp["j"], sys.op(cp["j"], cp["op_j"]), t), cp["j"], dims)
        V += cp["g"] * (A @ B)
        dcoup.append(A @ B)
    return V, dpar, dcoup


def jumps(sys, t):
    """Unit-rate jump operators of every mode in the interaction picture:
    [(mode, a_m(t), n_m)], each embedded; the rates multiply them."""
    out = []
    for m, d in enumerate(sys.dims):
        a = embed(sys.rotated(m, ladder(d), t), m, sys.dims)
        nm = embed(number(d), m, sys.dims)
        out.append((m, a, nm))
    return out


def dissipator(L, rho):
    """L rho L^dag - 1/2 {L^dag L, rho} for a stack rho (S, D, D)."""
    LdL = L.conj().T @ L
    return L @ rho @ L.conj().T - 0.5 * (LdL @ rho + rho @ LdL)


def dissipator_adj(L, X):
    """Adjoint of dissipator under <A, B> = tr(A^dag B)."""
    LdL = L.conj().T @ L
    return L.conj().T @ X @ L - 0.5 * (LdL @ X + X @ LdL)


def rhs(sys, g1, gp, n, s, rho):
    """d rho_I/dt at RK4 stage s of step n (rho: (S, D, D))."""
    V, _, _ = generator(sys, n, s)
    out = -1j * (V @ rho - rho @ V)
    for m, a, nm in jumps(sys, sys.stage_time(n, s)):
        if g1[m] != 0.0:
            out += g1[m] * dissipator(a, rho)
        if gp[m] != 0.0:
            out += 2.0 * gp[m] * dissipator(nm, rho)
    return out


def rhs_adj(sys, g1, gp, n, s, X):
    V, _, _ = generator(sys, n, s)
    out = 1j * (V @ X - X @ V)
    for m, a, nm in jumps(sys, sys.stage_time(n, s)):
        if g1[m] != 0.0:
            out += g1[m] * dissipator_adj(a, X)
        if gp[m] != 0.0:
            out += 2.0 * gp[m] * dissipator_adj(nm, X)
    return out


def rk4_step(sys, g1, gp, n, rho, keep_stages=False):
    h = sys.h
    y1 = rho
    k1 = rhs(sys, g1, gp, n, 0, y1)
    y2 = rho + 0.5 * h * k1
    k2 = rhs(sys, g1, gp, n, 1, y2)
    y3 = rho + 0.5 * h * k2
    k3 = rhs(sys, g1, gp, n, 2, y3)
    y4 = rho + h * k3
    k4 = rhs(sys, g1, gp, n, 3, y4)
    new = rho + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    if keep_stages:
        return new, (y1, y2, y3, y4)
    return new


def propagate(sys, rho0, g1=None, gp=None, n_steps=None):
    """rho_I(T) for a stack of initial matrices rho0 (S, D, D)."""
    if g1 is None:
        g1, gp = rates(sys.desc)
    rho = np.array(rho0, dtype=np.complex128)
    N = sys.N if n_steps is None else n_steps
    for n in range(N):
        rho = rk4_step(sys, g1, gp, n, rho)
    return rho


def input_states(desc):
    """Basis indices of the computational input states."""
    return [desc["columns"][c] for c in desc["comp_cols"]]


def matrix_units(D, states):
    """E_ab = |s_a><s_b| for the input states, stacked in the order j = a dc + b."""
    dc = len(states)
    out = np.zeros((dc * dc, D, D), dtype=np.complex128)
    for a in range(dc):
        for b in range(dc):
            out[a * dc + b, states[a], states[b]] = 1.0
    return out


def channel_overlap(rhoT, comp_rows, target):
    """sum_ab <u_a| rho_ab(T) |u_b>, rho_ab the image of E_ab (order a dc + b)."""
    dc = len(comp_rows)
    T = np.asarray(target, dtype=np.complex128)
    rows = list(comp_rows)
    tot = 0.0 + 0.0j
    for a in range(dc):
        for b in range(dc):
            blk = rhoT[a * dc + b][np.ix_(rows, rows)]
            tot += np.conj(T[:, a]) @ blk @ T[:, b]
    return complex(tot)


def average_fidelity(rhoT, comp_rows, target):
    dc = len(comp_rows)
    ov = channel_overlap(rhoT, comp_rows, target)
    return (ov.real + dc) / (dc * (dc + 1.0)), ov


def channel_cotangent(shape, comp_rows, target):
    """lambda with dLoss = 2 Re <lambda, d rho(T)> for Loss = 1 - F:
    lambda_ab[r_i, r_j] = -T_ia conj(T_jb) / (2 dc (dc + 1))."""
    dc = len(comp_rows)
    T = np.asarray(target, dtype=np.complex128)
    lam = np.zeros(shape, dtype=np.complex128)
    rows = list(comp_rows)
    c = -1.0 / (2.0 * dc * (dc + 1.0))
    for a in range(dc):
        for b in range(dc):
            lam[a * dc + b][np.ix_(rows, rows)] = c * np.outer(T[:, a], np.conj(T[:, b]))
    return lam


def param_names(sys):
    names = []
    for k, dr in enumerate(sys.drives):
        for p in range(len(dr["params"])):
            names.append(f"drive{k}.p{p}")
    for e in range(len(sys.couplings)):
        names.append(f"coupling{e}.g")
    for m in range(sys.n_modes):
        names += [f"mode{m}.gamma1", f"mode{m}.gammaphi"]
    return names


def _inner(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def _stage_grad(sys, g1, gp, n, s, kb, y, grad):
    """grad += 2 Re <kb, dL_s/dtheta y> for every parameter."""
    V, dpar, dcoup = generator(sys, n, s)
    i = 0
    for O in dpar + dcoup:
        grad[i] += 2.0 * _inner(kb, -1j * (O @ y - y @ O)).real
        i += 1
    for m, a, nm in jumps(sys, sys.stage_time(n, s)):
        grad[i] += 2.0 * _inner(kb, dissipator(a, y)).real
        grad[i + 1] += 2.0 * _inner(kb, 2.0 * dissipator(nm, y)).real
        i += 2


def gradient(sys, lam_T, rho0, g1=None, gp=None):
    """dLoss/dtheta given the cotangent lam_T of rho(T) (stored forward states)."""
    if g1 is None:
        g1, gp = rates(sys.desc)
    h = sys.h
    states = [np.array(rho0, dtype=np.complex128)]
    for n in range(sys.N):
        states.append(rk4_step(sys, g1, gp, n, states[-1]))
    grad = np.zeros(len(param_names(sys)))
    lam = np.array(lam_T, dtype=np.complex128)
    for n in reversed(range(sys.N)):
        _, ys = rk4_step(sys, g1, gp, n, states[n], keep_stages=True)
        kb4 = (h / 6.0) * lam
        yb4 = rhs_adj(sys, g1, gp, n, 3, kb4)
        kb3 = (h / 3.0) * lam + h * yb4
        yb3 = rhs_adj(sys, g1, gp, n, 2, kb3)
        kb2 = (h / 3.0) * lam + 0.5 * h * yb3
        yb2 = rhs_adj(sys, g1, gp, n, 1, kb2)
        kb1 = (h / 6.0) * lam + 0.5 * h * yb2
        yb1 = rhs_adj(sys, g1, gp, n, 0, kb1)
        for s, kb in enumerate((kb1, kb2, kb3, kb4)):
            _stage_grad(sys, g1, gp, n, s, kb, ys[s], grad)
        lam = lam + yb1 + yb2 + yb3 + yb4
    return grad


def loss_and_grad(sys, g1=None, gp=None):
    """Loss 1 - F of the channel on the computational subspace and its gradient."""
    desc = sys.desc
    if g1 is None:
        g1, gp = rates(desc)
    rho0 = matrix_units(sys.D, input_states(desc))
    rhoT = propagate(sys, rho0, g1, gp)
    F, _ = average_fidelity(rhoT, desc["comp_rows"], desc["target"])
    lam = channel_cotangent(rhoT.shape, desc["comp_rows"], desc["target"])
    return 1.0 - F, gradient(sys, lam, rho0, g1, gp)
