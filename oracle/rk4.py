"""Fixed-step classical RK4 in the interaction picture (oracle; test only).

The time-ordered exponential U(0, T) = T exp(-i int H dt) (Sec. 2.3) is
approximated on the fixed grid t_n = n h, h = T/N (the product of step
propagators, Sec. 2.3) by classical RK4 applied to

    d psi_I/dt = -i V(t) psi_I,
    V(t) = exp(i H_f t) (H(t) - H_f) exp(-i H_f t),

where H_f = sum_m diag(eps^f_m) is the frame.  Because H_f is a sum of
single-mode diagonals, every local operator A_m keeps its Kronecker form and
only picks up phases, A_ab exp(i (eps^f_a - eps^f_b) t) (see system.py).
The product of a local operator with the state is a contraction of the rank-N
state tensor along one mode (App. B); here numpy.tensordot does it.

The returned state is psi_I(T) = exp(i H_f T) psi_lab(T).
"""
from __future__ import annotations

import math

import numpy as np


def apply_op(op, m, psi):
    """(I (x) .. op on mode m .. (x) I) psi for psi shaped dims + (S,)."""
    out = np.tensordot(op, psi, axes=([1], [m]))
    return np.moveaxis(out, 0, m)


def apply_diag(vals, m, psi):
    shape = [1] * psi.ndim
    shape[m] = len(vals)
    return vals.reshape(shape) * psi


def apply_generator(sys, n, s, psi):
    """V(t) psi at RK4 stage s of step n, one local term at a time."""
    t = sys.stage_time(n, s)
    out = np.zeros_like(psi)
    for m in range(sys.n_modes):
        dl = sys.delta(m)
        if np.any(dl != 0.0):
            out += apply_diag(dl.astype(np.complex128), m, psi)
    for c in sys.couplings:
        A = sys.rotated(c["i"], sys.op(c["i"], c["op_i"]), t)
        B = sys.rotated(c["j"], sys.op(c["j"], c["op_j"]), t)
        out += c["g"] * apply_op(B, c["j"], apply_op(A, c["i"], psi))
    for k, dr in enumerate(sys.drives):
        ck, _ = sys.drive_coeff(k, n, s)
        O = sys.rotated(dr["mode"], sys.op(dr["mode"], dr["op"]), t)
        out += ck * apply_op(O, dr["mode"], psi)
    return out


def rk4_step(sys, n, psi, keep_stages=False):
    """One classical RK4 step (nodes 0, h/2, h/2, h; weights 1/6, 1/3, 1/3, 1/6)."""
    h = sys.h
    y1 = psi
    k1 = -1j * apply_generator(sys, n, 0, y1)
    y2 = psi + (0.5 * h) * k1
    k2 = -1j * apply_generator(sys, n, 1, y2)
    y3 = psi + (0.5 * h) * k2
    k3 = -1j * apply_generator(sys, n, 2, y3)
    y4 = psi + h * k3
    k4 = -1j * apply_generator(sys, n, 3, y4)
    new = psi + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    if keep_stages:
        return new, (y1, y2, y3, y4)
    return new


def as_tensor(sys, psi):
    psi = np.asarray(psi, dtype=np.complex128)
    return psi.reshape(sys.dims + [psi.shape[1]])


def basis_columns(D, columns):
    psi0 = np.zeros((D, len(columns)), dtype=np.complex128)
    for j, c in enumerate(columns):
        psi0[c, j] = 1.0
    return psi0


def propagate(sys, psi0=None, ckpt_every=None, n_steps=None):
    """Propagate the columns psi0 (D, S) over all steps.

    Returns psi_I(T) as (D, S); with ``ckpt_every`` also the list of states at
    steps 0, c, 2c, ... (as tensors)."""
    if psi0 is None:
        psi0 = basis_columns(sys.D, sys.desc["columns"])
    S = psi0.shape[1]
    psi = as_tensor(sys, psi0)
    N = sys.N if n_steps is None else n_steps
    ckpts = []
    for n in range(N):
        if ckpt_every and n % ckpt_every == 0:
            ckpts.append(psi.copy())
        psi = rk4_step(sys, n, psi)
    out = psi.reshape(sys.D, S)
    if ckpt_every:
        return out, ckpts
    return out


def default_ckpt(N):
    return int(math.ceil(math.sqrt(N)))
