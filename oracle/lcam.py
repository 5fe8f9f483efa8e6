"""Local continuous adjoint method (LCAM) of the product formulas (oracle;
test infrastructure only).

Sec. 2.5 (continuous adjoint method): the gradient of a loss of the final
state is a sum over the step factors of a_i^T (dU_i/dtheta) psi_{i-1} (eq. for
the i-th term), where the costate a_i is carried backward by the chain rule
a_i = U_{i+1}^T a_{i+1} and the states are recovered by evolving backward in
time instead of being stored.  With every step a product of local gates
(Sec. 2.3, App. A), dU_i/dtheta expands over those gates as in the eq. for
the derivative sum, so each gate contributes through a local derivative only
(the "local" part of the method).  Here the walk is done gate by gate:

    phi  = G^-1 psi          (the state before the gate, recovered backward)
    dL  += 2 Re <mu, (dG/dtheta) phi>
    mu  <- G^dag mu          (the costate before the gate)
    psi <- phi

with complex states and the convention dL = 2 Re <lambda, d psi>,
lambda = dL/d psi* (the real-vector transpose of the paper becomes the
adjoint).  For a gate G = exp(X), X = -i a tau h, with h its local term,
dG = L(X, dX) is the Frechet derivative of the matrix exponential, taken
from the block-triangular exponential expm([[X, E], [0, X]]) =
[[e^X, L(X, E)], [0, e^X]] (Van Loan 1978; Najfeld and Havel 1995).  With
M_ab = sum_rest conj(mu[a, rest]) phi[b, rest] the gate's local reduced
matrix, sum_ab dG_ab M_ab = Tr(M^T L(X, dX)) = Tr(L(X, M^T) dX) (the
Frechet derivative of exp is symmetric under the trace pairing), so every
parameter of the gate needs only K = L(X, M^T) and its dh/dtheta:
dL += 2 Re(-i a tau Tr(K dh/dtheta)).

Parameters and their local derivatives, at the frozen time of the gate:
  drive k parameter p:   single-mode term of its mode, dh = dc_k/dp O_k
  (E_J, E_C, E_L) of m:  single-mode term, dh = diag(d eps_m) + sum_k c_k dO_k;
                         coupling terms on m, g (dA (x) B) or g (A (x) dB)
  coupling g_e:          its two-body term, dh = A (x) B
The frame and the carriers are held fixed (the frame rotation of the output,
exp(i H_f T), does not depend on the parameters).  For Q4j the gates are not
unitary: the state is recovered with G^-1 = exp(-X), the costate uses G^dag.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from .adjoint import DEV
from .rk4 import as_tensor
from .trotter import coefficients, drive_value, local_terms, midpoints, to_frame, \
    trotter_step, apply_local


def frechet_exp(X, E):
    """L(X, E), the Frechet derivative of exp at X in the direction E."""
    n = X.shape[0]
    Z = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    Z[:n, :n] = X
    Z[n:, n:] = X
    Z[:n, n:] = E
    return expm(Z)[:n, n:]


def local_reduced(mu, phi, modes):
    """M_ab = sum over every other index (columns included) of
    conj(mu[a, rest]) phi[b, rest]; a, b run over the gate's local indices in
    the order of ``modes`` (for two modes: digit of modes[0] * d + digit of
    modes[1])."""
    k = len(modes)
    mu2 = np.moveaxis(mu, list(modes), list(range(k)))
    ph2 = np.moveaxis(phi, list(modes), list(range(k)))
    loc = int(np.prod(mu2.shape[:k]))
    a = mu2.reshape(loc, -1)
    b = ph2.reshape(loc, -1)
    return np.conj(a) @ b.T


def _term_derivatives(sys, n, t, term_index):
    """[(param index, dh)] of local term ``term_index`` (order of
    trotter.local_terms) at time t of step n."""
    out = []
    M = sys.n_modes
    npulse = sum(len(dr["params"]) for dr in sys.drives)
    if term_index < M:
        m = term_index
        idx = 0
        for k, dr in enumerate(sys.drives):
            if dr["mode"] == m:
                _, de = sys.envelope(dr, n, t)
                cr = np.cos(dr["omega_d"] * t + dr["phase"])
                O = sys.op(m, dr["op"])
                for p in range(len(de)):
                    out.append((idx + p, de[p] * cr * O))
            idx += len(dr["params"])
        mode = sys.modes[m]
        for p, name in enumerate(DEV):
            dh = np.diag(mode["deps"][name]).astype(np.complex128)
            for k, dr in enumerate(sys.drives):
                if dr["mode"] == m:
                    dh = dh + drive_value(sys, k, n, t) * mode["dops"][name][dr["op"]]
            out.append((npulse + 3 * m + p, dh))
        return out
    e = term_index - M
    c = sys.couplings[e]
    A = sys.op(c["i"], c["op_i"])
    B = sys.op(c["j"], c["op_j"])
    out.append((npulse + 3 * M + e, np.kron(A, B)))
    for p, name in enumerate(DEV):
        dA = sys.modes[c["i"]]["dops"][name][c["op_i"]]
        dB = sys.modes[c["j"]]["dops"][name][c["op_j"]]
        out.append((npulse + 3 * c["i"] + p, c["g"] * np.kron(dA, B)))
        out.append((npulse + 3 * c["j"] + p, c["g"] * np.kron(A, dB)))
    return out


def gradient(sys, order, lam_T, psi0):
    """dL/dtheta by LCAM for the costate lam_T (D, S) of psi_I(T), the columns
    psi0 (D, S) propagated by the product formula ``order``.  Only the final
    state of the forward is kept; the walk back recovers every earlier state."""
    S = psi0.shape[1]
    N = sys.N
    psi = as_tensor(sys, psi0)
    for n in range(N):
        psi = trotter_step(sys, n, psi, order)
    mu = to_frame(sys, as_tensor(sys, lam_T), -N * sys.h)   # exp(-i H_f T) lambda_I
    grad = np.zeros(sys.n_params())
    a, symmetric = coefficients(order)
    dt = sys.h
    tau = 0.5 * dt if symmetric else dt
    for n in range(N - 1, -1, -1):
        t_n = n * dt
        pieces = list(zip(a, midpoints(order, dt)))
        for aj, mid in reversed(pieces):
            t = t_n + mid
            terms = local_terms(sys, n, t)
            seq = list(range(len(terms)))
            if symmetric:
                seq = seq + seq[::-1]
            for ti in reversed(seq):
                modes, H = terms[ti]
                X = -1j * aj * tau * H
                phi = apply_local(expm(-X), modes, psi)
                Mred = local_reduced(mu, phi, modes)
                K = frechet_exp(X, Mred.T)
                for pidx, dh in _term_derivatives(sys, n, t, ti):
                    grad[pidx] += 2.0 * (-1j * aj * tau * np.trace(K @ dh)).real
                mu = apply_local(expm(X).conj().T, modes, mu)
                psi = phi
    return grad
