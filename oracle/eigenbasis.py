"""Multi-qubit eigenbasis transform and local-unitary compensation of the
fidelity (oracle; test infrastructure only).

App. D (details of time evolution): the time evolution runs in the product
basis, and the final unitary is expressed in the eigenbasis of the idling
(static) Hamiltonian, U -> V^dag U V (eq. for the basis transform), by
evolving the initial states V|psi> in the product basis and projecting the
final ones with V^dag.  The eigenstates are the columns of V after "adjusting
the phases of its eigenstates".  Readings:
  - the idling Hamiltonian is the static one of the spectrum oracle,
    H0 = sum_m diag(eps_m) + sum_e g_e A_i (x) B_j in the dressed single-mode
    bases; the eigenstate of computational state k is the eigenvector with the
    largest overlap |<k|v>|^2 with the bare product state k (the labelling of
    the energy tensor, Sec. 3.2);
  - its phase is fixed by making <k|v> real and positive;
  - the eigenbasis unitary is taken in the frame of the dressed energies E_k
    (each eigenstate rotating at its own energy), the eigenbasis analogue of
    the product-frame interaction picture: M_ij = exp(i E_i T) <v_i| U_lab |v_j>;
  - the basis and the energies are those of the nominal parameters, held
    fixed when parameters move (as the frame energies are).
With psi_I(T) = exp(i H_f T) U_lab psi(0) (the propagated frame),
M_ij = <w_i | psi_I,j(T)> with w_i = exp(i (H_f - E_i) T) v_i, so the
eigenbasis gate fidelity |Tr(T^dag M)|^2 / d_c^2 is the composite state cost
(Sec. 4.1) of the columns psi(0) = v_j against the target states
phi_j = sum_i T_ij w_i.

Compensation (App. D step 6): error-free single-qubit gates before and after
the simulated gate align it with the target.  With arbitrary single-qubit
unitaries (the SU(2) per qubit form of the paper's SU(4) for two qubits),
F = max |Tr(T^dag (x)_q a_q  M  (x)_q b_q)|^2 / d_c^2 over unitaries a_q
(after) and b_q (before).  The maximum is sought by coordinate ascent from the
identity: with the others fixed, tau is linear in one a_q (or b_q),
tau = Tr(a_q X), and |Tr(a X)| over unitaries a is largest, equal to the sum
of the singular values of X, at a = Q P^dag for X = P S Q^dag (the polar
factor; von Neumann's trace inequality).  Sweeps over a_0..a_{n-1}, then
b_0..b_{n-1} repeat until |tau| grows by at most tol (relative).  The
search is local: it reaches the maximum for the targets the compensation is
meant for (CZ, CNOT, products of single-qubit gates) and can stop below it
for generic entangling targets.  At the
optimum the gates are stationary, so the compensated loss has the plain
loss's cotangent with the compensated target T' = A^dag T B^dag.
"""
from __future__ import annotations

import numpy as np

from .spectrum import static_hamiltonian


def frame_diagonal(sys):
    """H_f on the product basis: f(k) = sum_m frame_m[digit_m(k)]."""
    f = np.zeros(1)
    for m in range(sys.n_modes):
        f = (f[:, None] + sys.frame[m][None, :]).reshape(-1)
    return f


def dressed_states(sys, labels):
    """(V_c, E_c): for each bare index in ``labels`` its dressed eigenstate
    (column, phase fixed so that <k|v> > 0) and energy."""
    H = static_hamiltonian(sys)
    w, V = np.linalg.eigh(H)
    cols, E = [], []
    for k in labels:
        v_idx = int(np.argmax(np.abs(V[k, :]) ** 2))
        v = V[:, v_idx].astype(np.complex128)
        v = v * (np.conj(v[k]) / abs(v[k]))
        cols.append(v)
        E.append(w[v_idx])
    return np.array(cols).T, np.array(E)


def eigenbasis_targets(sys, labels, target, T):
    """(psi0, phi): the initial states v_j and the target states
    phi_j = sum_i T_ij w_i, w_i = exp(i (H_f - E_i) T) v_i."""
    Vc, Ec = dressed_states(sys, labels)
    f = frame_diagonal(sys)
    W = np.exp(1j * (f[:, None] - Ec[None, :]) * T) * Vc
    return Vc, W @ np.asarray(target, dtype=np.complex128), W


def _apply_local(mats, n, M, side):
    """(x)_q mats[q] times M (side 0, from the left) or M times it (side 1),
    qubit 0 most significant."""
    K = np.ones((1, 1), dtype=np.complex128)
    for q in range(n):
        K = np.kron(K, mats[q])
    return K @ M if side == 0 else M @ K


def local_tau(M, target, a, b):
    """tau = Tr(T^dag (x)a  M  (x)b)."""
    n = len(a)
    X = _apply_local(b, n, _apply_local(a, n, M, 0), 1)
    return complex(np.trace(np.conj(np.asarray(target)).T @ X))


def _partial(Y, n, q):
    """X_q with Tr(a_q X_q) = Tr((I (x) .. a_q .. (x) I) Y): the partial trace of
    Y over every qubit but q."""
    t = Y.reshape([2] * (2 * n))
    # contract every other qubit's row index with its column index
    rest = [p for p in range(n) if p != q]
    for p in sorted(rest, reverse=True):
        t = np.trace(t, axis1=p, axis2=p + t.ndim // 2)
    # t[r, c] = sum_rest Y[(r, rest), (c, rest)], and Tr(a t) = sum a[c, r] t[r, c]
    return t


def su2_fidelity(M, target, n_q, max_sweeps=500, tol=1e-14):
    """(F, a, b, tau): the fidelity with arbitrary single-qubit unitaries
    before (b) and after (a) the gate, by coordinate ascent from identities."""
    M = np.asarray(M, dtype=np.complex128)
    T = np.asarray(target, dtype=np.complex128)
    dc = 2 ** n_q
    assert M.shape == (dc, dc) and T.shape == (dc, dc)
    a = [np.eye(2, dtype=np.complex128) for _ in range(n_q)]
    b = [np.eye(2, dtype=np.complex128) for _ in range(n_q)]
    best = abs(local_tau(M, T, a, b))
    Th = np.conj(T).T
    for _ in range(max_sweeps):
        for side in (0, 1):
            for q in range(n_q):
                if side == 0:
                    # tau = Tr((x)a M B T^dag): the matrix multiplying (x)a
                    rest = [np.eye(2) if p == q else a[p] for p in range(n_q)]
                    Y = _apply_local(rest, n_q, _apply_local(b, n_q, M, 1) @ Th, 0)
                else:
                    # tau = Tr((x)b T^dag A M)
                    rest = [np.eye(2) if p == q else b[p] for p in range(n_q)]
                    Y = _apply_local(rest, n_q, Th @ _apply_local(a, n_q, M, 0), 0)
                X = _partial(Y, n_q, q)
                P, s, Qh = np.linalg.svd(X)
                u = np.conj(Qh).T @ np.conj(P).T     # Tr(u X) = sum s
                if side == 0:
                    a[q] = u
                else:
                    b[q] = u
        t = abs(local_tau(M, T, a, b))
        done = t - best <= tol * max(1.0, t)
        best = max(best, t)
        if done:
            break
    tau = local_tau(M, T, a, b)
    return abs(tau) ** 2 / dc ** 2, a, b, tau


def su2_target(target, a, b):
    """T' = A^dag T B^dag with A = (x)a, B = (x)b: at the optimum the
    compensated loss has the plain cotangent with T'."""
    n = len(a)
    T = np.asarray(target, dtype=np.complex128)
    A = np.ones((1, 1), dtype=np.complex128)
    B = np.ones((1, 1), dtype=np.complex128)
    for q in range(n):
        A = np.kron(A, a[q])
        B = np.kron(B, b[q])
    return np.conj(A).T @ T @ np.conj(B).T
