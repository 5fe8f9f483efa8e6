"""Gate fidelity on the computational subspace (oracle; test only).

F = |Tr(U_t^dag P U P)|^2 / d_c^2: the composite state-transfer cost of
Sec. 4.1 (eq. for the composite state cost) with the S = d_c columns of the
target as target states, L = 1 - F.  For a unitary channel the average gate
fidelity of App. D (eq. for the average fidelity) is (d_c F + 1)/(d_c + 1).

Cotangent: with the convention dL = 2 Re <lambda, dU> (<a,b> = sum conj(a) b),
lambda[comp_i, col_j] = -(tau / d_c^2) T_ij and zero elsewhere, where
tau = sum_ij conj(T_ij) U[comp_i, col_j].
"""
from __future__ import annotations

import numpy as np


def overlap(U, comp_rows, comp_cols, target):
    P = np.asarray(U)[np.ix_(list(comp_rows), list(comp_cols))]
    return complex(np.sum(np.conj(target) * P))


def fidelity(U, comp_rows, comp_cols, target):
    dc = len(comp_rows)
    tau = overlap(U, comp_rows, comp_cols, target)
    return abs(tau) ** 2 / dc ** 2, tau


def average_gate_fidelity(F, dc):
    return (dc * F + 1.0) / (dc + 1.0)


def cotangent(shape, comp_rows, comp_cols, target, tau):
    dc = len(comp_rows)
    lam = np.zeros(shape, dtype=np.complex128)
    for i, r in enumerate(comp_rows):
        for j, c in enumerate(comp_cols):
            lam[r, c] = -(tau / dc ** 2) * target[i, j]
    return lam


def comp_bits(n_q):
    """bits[i, q] = bit of qubit q in computational index i (qubit 0 most
    significant, the binary order of the computational states)."""
    dc = 2 ** n_q
    return np.array([[(i >> (n_q - 1 - q)) & 1 for q in range(n_q)] for i in range(dc)],
                    dtype=np.int64)


def zcomp_overlap(M, target, a, c):
    """tau(a, c) = sum_ij conj(T_ij) e^{i theta_i} M_ij e^{i chi_j} with
    theta_i = sum_q a_q bit_q(i) (phases after the gate) and chi_j = sum_q c_q
    bit_q(j) (phases before it)."""
    bits = comp_bits(len(a))
    th = bits @ np.asarray(a, dtype=np.float64)
    ch = bits @ np.asarray(c, dtype=np.float64)
    W = np.conj(target) * M
    return complex(np.sum(np.exp(1j * th)[:, None] * W * np.exp(1j * ch)[None, :]))


ZC_GOLDEN = 0.6180339887498949   # fractional part of the golden ratio


def zcomp_starts(n_q):
    """Starting phases of the multi-start search: 1 start (zero) for one
    qubit, 16 otherwise; start k has a_q = 2 pi frac(k (q + 1) g) and
    c_q = 2 pi frac(k (n_q + q + 1) g), g = ZC_GOLDEN (start 0 is zero)."""
    K = 1 if n_q == 1 else 16
    out = []
    for k in range(K):
        a = np.array([2 * np.pi * ((k * (q + 1) * ZC_GOLDEN) % 1.0) for q in range(n_q)])
        c = np.array([2 * np.pi * ((k * (n_q + q + 1) * ZC_GOLDEN) % 1.0) for q in range(n_q)])
        out.append((a, c))
    return out


def _zcomp_ascend(W, bits, a, c, max_sweeps, tol):
    """Coordinate ascent from (a, c): in turn a_0..a_{n-1}, then
    c_0..c_{n-1}, each phase set to its optimum with the others fixed.  With
    tau = A + e^{i p} B, B the terms whose bit of that qubit is set, |tau| is
    largest at p = arg A - arg B (a phase whose A or B vanishes is left as it
    is).  Sweeps repeat until |tau| grows by at most tol (relative) or
    max_sweeps is reached."""
    n_q = bits.shape[1]
    a = np.array(a, dtype=np.float64)
    c = np.array(c, dtype=np.float64)

    def tau_of(a, c):
        return (np.exp(1j * (bits @ a))[:, None] * W * np.exp(1j * (bits @ c))[None, :]).sum()

    best = abs(tau_of(a, c))
    for _ in range(max_sweeps):
        for side in (0, 1):
            for q in range(n_q):
                th = bits @ a
                ch = bits @ c
                if side == 0:
                    th = th - a[q] * bits[:, q]
                    X = np.exp(1j * th)[:, None] * W * np.exp(1j * ch)[None, :]
                    A = X[bits[:, q] == 0, :].sum()
                    B = X[bits[:, q] == 1, :].sum()
                else:
                    ch = ch - c[q] * bits[:, q]
                    X = np.exp(1j * th)[:, None] * W * np.exp(1j * ch)[None, :]
                    A = X[:, bits[:, q] == 0].sum()
                    B = X[:, bits[:, q] == 1].sum()
                if A != 0 and B != 0:
                    p = np.angle(A) - np.angle(B)
                    if side == 0:
                        a[q] = p
                    else:
                        c[q] = p
        t = abs(tau_of(a, c))
        done = t - best <= tol * max(1.0, t)
        best = max(best, t)
        if done:
            break
    return a, c


def zcomp_fidelity(M, target, n_q, max_sweeps=200, tol=1e-14):
    """Fidelity with error-free single-qubit phase gates before and after the
    gate (the compensation of App. D, restricted to Z rotations: virtual Z),
    F = max_{a,c} |tau(a, c)|^2 / d_c^2 for the d_c x d_c computational block
    M.  The maximum is sought by coordinate ascent (_zcomp_ascend) from each
    start of zcomp_starts; the start reaching the largest |tau| wins (the
    earliest on a tie).  Returns (F, a, c, tau)."""
    M = np.asarray(M, dtype=np.complex128)
    target = np.asarray(target, dtype=np.complex128)
    dc = 2 ** n_q
    assert M.shape == (dc, dc) and target.shape == (dc, dc)
    bits = comp_bits(n_q)
    W = np.conj(target) * M
    best = None
    for a0, c0 in zcomp_starts(n_q):
        a, c = _zcomp_ascend(W, bits, a0, c0, max_sweeps, tol)
        t = abs(zcomp_overlap(M, target, a, c))
        if best is None or t > best[0]:
            best = (t, a, c)
    _, a, c = best
    tau = zcomp_overlap(M, target, a, c)
    return abs(tau) ** 2 / dc ** 2, a, c, tau


def zcomp_target(target, a, c):
    """The target rephased by the optimal phases, T'_ij = T_ij e^{-i theta_i}
    e^{-i chi_j}: at the optimum the compensated loss has the plain loss's
    cotangent with T' (the phases are stationary, so they carry no
    derivative)."""
    bits = comp_bits(len(a))
    th = bits @ np.asarray(a, dtype=np.float64)
    ch = bits @ np.asarray(c, dtype=np.float64)
    return np.asarray(target) * np.exp(-1j * th)[:, None] * np.exp(-1j * ch)[None, :]


def state_fidelity(U, targets):
    """Composite state-transfer cost of Sec. 4.1 (eq. for the composite state
    cost): F = |(1/S) sum_s <phi_s|psi_s>|^2 and L = 1 - F, where psi_s are the
    S columns of U (D x S) and phi_s the columns of ``targets`` (D x S), full
    target states rather than a computational block.  Returns (F, tau) with
    tau = sum_s <phi_s|psi_s>."""
    U = np.asarray(U)
    targets = np.asarray(targets)
    assert U.shape == targets.shape
    S = U.shape[1]
    tau = complex(np.sum(np.conj(targets) * U))
    return abs(tau) ** 2 / S ** 2, tau


def state_cotangent(targets, tau):
    """Costate of the composite state cost with dL = 2 Re <lambda, dU>:
    dL = -2 Re(conj(tau) <phi, dU>) / S^2, so lambda = -(tau / S^2) phi."""
    targets = np.asarray(targets, dtype=np.complex128)
    S = targets.shape[1]
    return -(tau / S ** 2) * targets
