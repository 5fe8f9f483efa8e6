"""Discrete adjoint of the RK4 propagation (oracle; test only).

The gradient is the sum over steps of the per-step terms of Sec. 2.5
(eqs. for the derivative sum and its i-th term): the costate is carried
backward through the chain rule a_i = U_{i+1}^T a_{i+1}, where U_{i+1} is
here one RK4 step, and each step contributes the derivative of that step map
w.r.t. theta applied to the stored forward state.  For complex states the
convention is dL = 2 Re <lambda, d psi>.

For one step psi' = psi + h/6 (k1 + 2 k2 + 2 k3 + k4), k_s = A_s y_s,
A_s = -i V(t_s) (so A_s^dag = i V(t_s)), the reverse map from lambda' is

    kb4 = h/6 lambda'            yb4 = A4^dag kb4
    kb3 = h/3 lambda' + h yb4     yb3 = A3^dag kb3
    kb2 = h/3 lambda' + h/2 yb3   yb2 = A2^dag kb2
    kb1 = h/6 lambda' + h/2 yb2   yb1 = A1^dag kb1
    lambda = lambda' + yb1 + yb2 + yb3 + yb4
    dL/dtheta += 2 Re <kb_s, dA_s/dtheta y_s> = 2 Im <kb_s, dV_s/dtheta y_s>.

States are recomputed segment by segment from checkpoints taken every
ceil(sqrt(N)) steps.  Derivatives of V w.r.t. every parameter are applied
term by term: drive parameters through dc_k/dp, couplings through their
operator product, device parameters (E_J, E_C, E_L) through d eps and the
dressed-operator derivatives of single_mode.mode_derivatives; the frame and
the carriers are held fixed.

Parameter order: drive parameters (drive order, then parameter order), then
(E_J, E_C, E_L) of every mode, then the coupling strengths.
"""
from __future__ import annotations

import numpy as np

from .fidelity import cotangent, fidelity
from .rk4 import apply_diag, apply_generator, apply_op, as_tensor, basis_columns, \
    default_ckpt, propagate, rk4_step

DEV = ("EJ", "EC", "EL")


def param_names(sys):
    names = []
    for k, dr in enumerate(sys.drives):
        for p in range(len(dr["params"])):
            names.append(f"drive{k}.p{p}")
    for m in range(sys.n_modes):
        for p in DEV:
            names.append(f"mode{m}.{p}")
    for e in range(len(sys.couplings)):
        names.append(f"coupling{e}.g")
    return names


def _inner(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def _stage_grad(sys, n, s, kb, y, grad):
    """Accumulate 2 Im <kb, dV/dtheta y> for every parameter at stage s."""
    t = sys.stage_time(n, s)
    idx = 0
    # drive parameters
    for k, dr in enumerate(sys.drives):
        O = sys.rotated(dr["mode"], sys.op(dr["mode"], dr["op"]), t)
        ov = _inner(kb, apply_op(O, dr["mode"], y))
        _, dc = sys.drive_coeff(k, n, s)
        for p in range(len(dc)):
            grad[idx + p] += 2.0 * (dc[p] * ov).imag
        idx += len(dc)
    # device parameters
    for m in range(sys.n_modes):
        mode = sys.modes[m]
        for p in DEV:
            dV_y = apply_diag(mode["deps"][p].astype(np.complex128), m, y)
            for c in sys.couplings:
                if c["i"] == m or c["j"] == m:
                    A = sys.rotated(c["i"], sys.op(c["i"], c["op_i"]), t)
                    B = sys.rotated(c["j"], sys.op(c["j"], c["op_j"]), t)
                    if c["i"] == m:
                        dA = sys.rotated(m, mode["dops"][p][c["op_i"]], t)
                        dV_y = dV_y + c["g"] * apply_op(B, c["j"], apply_op(dA, c["i"], y))
                    if c["j"] == m:
                        dB = sys.rotated(m, mode["dops"][p][c["op_j"]], t)
                        dV_y = dV_y + c["g"] * apply_op(dB, c["j"], apply_op(A, c["i"], y))
            for k, dr in enumerate(sys.drives):
                if dr["mode"] == m:
                    ck, _ = sys.drive_coeff(k, n, s)
                    dO = sys.rotated(m, mode["dops"][p][dr["op"]], t)
                    dV_y = dV_y + ck * apply_op(dO, m, y)
            grad[idx] += 2.0 * _inner(kb, dV_y).imag
            idx += 1
    # couplings
    for c in sys.couplings:
        A = sys.rotated(c["i"], sys.op(c["i"], c["op_i"]), t)
        B = sys.rotated(c["j"], sys.op(c["j"], c["op_j"]), t)
        grad[idx] += 2.0 * _inner(kb, apply_op(B, c["j"], apply_op(A, c["i"], y))).imag
        idx += 1


def reverse_step(sys, n, psi, lam_next, grad):
    """Adjoint of step n: psi is the state entering the step, lam_next the
    costate of the state leaving it.  Returns the costate entering it."""
    h = sys.h
    _, ys = rk4_step(sys, n, psi, keep_stages=True)
    Ad = lambda s, v: 1j * apply_generator(sys, n, s, v)   # A_s^dag
    kb4 = (h / 6.0) * lam_next
    yb4 = Ad(3, kb4)
    kb3 = (h / 3.0) * lam_next + h * yb4
    yb3 = Ad(2, kb3)
    kb2 = (h / 3.0) * lam_next + (0.5 * h) * yb3
    yb2 = Ad(1, kb2)
    kb1 = (h / 6.0) * lam_next + (0.5 * h) * yb2
    yb1 = Ad(0, kb1)
    for s, kb in enumerate((kb1, kb2, kb3, kb4)):
        _stage_grad(sys, n, s, kb, ys[s], grad)
    return lam_next + yb1 + yb2 + yb3 + yb4


def gradient(sys, lam_T, psi0=None, ckpt_every=None):
    """dL/dtheta given the costate lam_T (D, S) of the final state."""
    if psi0 is None:
        psi0 = basis_columns(sys.D, sys.desc["columns"])
    c = ckpt_every or default_ckpt(sys.N)
    _, ckpts = propagate(sys, psi0, ckpt_every=c)
    grad = np.zeros(sys.n_params())
    lam = as_tensor(sys, lam_T)
    n_seg = len(ckpts)
    for seg in range(n_seg - 1, -1, -1):
        start = seg * c
        stop = min(start + c, sys.N)
        states = [ckpts[seg]]
        for n in range(start, stop - 1):
            states.append(rk4_step(sys, n, states[-1]))
        for n in range(stop - 1, start - 1, -1):
            lam = reverse_step(sys, n, states[n - start], lam, grad)
    return grad, lam.reshape(sys.D, -1)


def loss_and_grad(sys, ckpt_every=None):
    """(L, F, tau, U_I(T), grad) for the system's columns and target."""
    d = sys.desc
    psi0 = basis_columns(sys.D, d["columns"])
    U = propagate(sys, psi0)
    F, tau = fidelity(U, d["comp_rows"], d["comp_cols"], d["target"])
    lam = cotangent(U.shape, d["comp_rows"], d["comp_cols"], d["target"], tau)
    grad, _ = gradient(sys, lam, psi0, ckpt_every)
    return 1.0 - F, F, tau, U, grad
