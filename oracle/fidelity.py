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
