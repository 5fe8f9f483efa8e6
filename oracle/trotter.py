"""Suzuki-Trotter product formulas in the lab frame (oracle; test infrastructure only).

Sec. 2.3 (Trotterization solver) and App. A (higher-order decompositions):
the step propagator U(t, t + dt) is replaced by a product of exponentials
of local terms H_k, each a one- or two-body operator, applied to the state
tensor one contraction at a time (App. B).

Local terms, in this fixed order (a reading: the paper does not list them):
  1. one single-mode term per mode m, in mode order,
        H_m(t) = diag(eps_m) + sum_{drives k on m} c_k(t) O_k,
  2. one two-body term per coupling e, in coupling order, g_e A_i (x) B_j.

Product formulas, each a sequence of sub-products Q2(a_j dt) or, for Q1,
one pass with coefficient 1:
  Q1:  exp(-i H_1 dt) ... exp(-i H_K dt)
  Q2:  sub-product with a = 1
  Q4:  a = (p, 1 - 2p, p), p = 1 / (2 - 2^(1/3))        (real fourth order)
  Q4j: a = (p, conj(p)),   p = 1/2 - i sqrt(3)/6       (complex fourth order)
where Q2(a dt) applies exp(-i a H_k dt/2) for k = 1..K and then for
k = K..1.  Readings where the paper is silent or garbled:
  - every written product is a sequence of actions in the order written
    (the first factor acts first);
  - the complex p of Q4j is printed garbled; it is read as
    p = (3 - i sqrt(3)) / 6, which satisfies p + conj(p) = 1 and
    p^3 + conj(p)^3 = 0, the order conditions of App. A;
  - Q4j as printed is two symmetric pieces; their product cancels the
    cubic term but keeps a commutator at dt^4 (p^2 != conj(p)^2), so it
    is third order globally, which the pins measure;
  - a time-dependent term is frozen at the middle of its sub-product:
    t_n + s_j + a_j dt / 2 with s_j = sum_{l<j} a_l dt for the real
    coefficients (Q1: the middle of the step).  A complex sub-step has no
    real middle; Q4j freezes both of its pieces at the middle of the step,
    t_n + dt / 2, which keeps it second order for driven terms (frozen at
    the real parts of the complex middles it would drop to first order).
    A piecewise-constant envelope takes the piece of the step index, as in
    the RK4 grid.
The lab frame keeps every factor unitary for real coefficients.  The
returned state is put in the frame of the RK4 path: psi_I(T) =
exp(i H_f T) psi_lab(T), with H_f = sum_m diag(eps^f_m).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm

from .rk4 import apply_op, as_tensor, basis_columns

P4 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
P4J = complex(0.5, -math.sqrt(3.0) / 6.0)
ORDERS = ("q1", "q2", "q4", "q4j")


def coefficients(order):
    """Sub-product coefficients a_j and whether each sub-product is the
    symmetric Q2 (False only for Q1)."""
    if order == "q1":
        return [1.0], False
    if order == "q2":
        return [1.0], True
    if order == "q4":
        return [P4, 1.0 - 2.0 * P4, P4], True
    if order == "q4j":
        return [P4J, P4J.conjugate()], True
    raise ValueError(order)


def midpoints(order, dt):
    """Offsets from t_n at which the local terms of each sub-product are frozen."""
    a, _ = coefficients(order)
    if order == "q4j":
        return [0.5 * dt for _ in a]
    out, s = [], 0.0
    for aj in a:
        out.append(s + 0.5 * aj * dt)
        s += aj * dt
    return out


def drive_value(sys, k, n, t):
    """c_k(t) = E(t) cos(omega_d t + phase) (App. C), at an arbitrary time."""
    dr = sys.drives[k]
    e, _ = sys.envelope(dr, n, t)
    return e * math.cos(dr["omega_d"] * t + dr["phase"])


def local_terms(sys, n, t):
    """[(modes, matrix)] of the local terms at time t of step n."""
    terms = []
    for m in range(sys.n_modes):
        H = np.diag(sys.modes[m]["eps"]).astype(np.complex128)
        for k, dr in enumerate(sys.drives):
            if dr["mode"] == m:
                H = H + drive_value(sys, k, n, t) * sys.op(m, dr["op"])
        terms.append(((m,), H))
    for c in sys.couplings:
        A = sys.op(c["i"], c["op_i"])
        B = sys.op(c["j"], c["op_j"])
        terms.append(((c["i"], c["j"]), c["g"] * np.kron(A, B)))
    return terms


def apply_local(G, modes, psi):
    """A one- or two-body operator on the state tensor (App. B contraction);
    for two modes the row index is (digit of modes[0]) * d + digit of modes[1]."""
    if len(modes) == 1:
        return apply_op(G, modes[0], psi)
    i, j = modes
    di, dj = psi.shape[i], psi.shape[j]
    G4 = G.reshape(di, dj, di, dj)
    out = np.tensordot(G4, psi, axes=([2, 3], [i, j]))
    return np.moveaxis(out, [0, 1], [i, j])


def trotter_step(sys, n, psi, order):
    """psi_lab(t_{n+1}) from psi_lab(t_n) by one product formula."""
    a, symmetric = coefficients(order)
    dt = sys.h
    t_n = n * dt
    for aj, mid in zip(a, midpoints(order, dt)):
        terms = local_terms(sys, n, t_n + mid)
        tau = 0.5 * dt if symmetric else dt
        gates = [(modes, expm(-1j * aj * tau * H)) for modes, H in terms]
        for modes, G in gates:
            psi = apply_local(G, modes, psi)
        if symmetric:
            for modes, G in reversed(gates):
                psi = apply_local(G, modes, psi)
    return psi


def to_frame(sys, psi, t):
    """exp(i H_f t) psi, H_f = sum_m diag(eps^f_m)."""
    for m in range(sys.n_modes):
        ph = np.exp(1j * sys.frame[m] * t)
        shape = [1] * psi.ndim
        shape[m] = len(ph)
        psi = ph.reshape(shape) * psi
    return psi


def propagate(sys, order, psi0=None, n_steps=None):
    """psi_I(T) (D, S) of the columns psi0 under the product formula."""
    if psi0 is None:
        psi0 = basis_columns(sys.D, sys.desc["columns"])
    S = psi0.shape[1]
    psi = as_tensor(sys, psi0)
    N = sys.N if n_steps is None else n_steps
    for n in range(N):
        psi = trotter_step(sys, n, psi, order)
    return to_frame(sys, psi, N * sys.h).reshape(sys.D, S)
