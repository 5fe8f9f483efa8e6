"""Pins of the eigenbasis-transform and local-unitary compensation oracle
(App. D) against facts it does not compute itself: the eigen-equation, the
product basis when nothing couples the modes, the exact idle evolution from a
dense matrix exponential, von Neumann's trace inequality for one qubit, exact
recovery of targets scrambled by local unitaries, the ordering against the
phase-only and plain fidelities, and the cotangent at the optimum against
central differences."""
import numpy as np
import pytest
from scipy.linalg import expm

import scp_inputs as si
from oracle import eigenbasis as eb
from oracle.fidelity import (cotangent, fidelity, state_fidelity, zcomp_fidelity)
from oracle.rk4 import basis_columns
from oracle.spectrum import static_hamiltonian
from oracle.system import OracleSystem


def _haar(n, rng):
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _ring():
    s = si.transmon_ring(si.rng_for(7, 3), 3, 3, 2.0, 10)
    return si._finish(s, [3] * 3, target=si.cz_target(3))


def test_dressed_states_solve_the_eigen_equation_with_fixed_phase():
    desc = _ring()
    o = OracleSystem(desc)
    V, E = eb.dressed_states(o, desc["comp_rows"])
    H = static_hamiltonian(o)
    assert np.abs(H @ V - V * E[None, :]).max() <= 1e-10 * np.abs(E).max()
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() <= 1e-12
    for j, k in enumerate(desc["comp_rows"]):
        assert abs(V[k, j].imag) <= 1e-15 and V[k, j].real > 0.5


def test_without_coupling_the_eigenbasis_is_the_product_basis():
    desc = _ring()
    for c in desc["couplings"]:
        c["g"] = 0.0
    o = OracleSystem(desc)
    T = _haar(8, np.random.default_rng(3))
    V, phi, W = eb.eigenbasis_targets(o, desc["comp_rows"], T, 1.7)
    B = basis_columns(o.D, desc["comp_rows"])
    assert np.abs(V - B).max() <= 1e-12
    # frame = the dressed single-mode energies, so w_i = e_i and phi = embedded T
    assert np.abs(phi - B @ T).max() <= 1e-12
    U = np.random.default_rng(4).normal(size=(o.D, 8)) + 0j
    F1, _ = state_fidelity(U, phi)
    F2, _ = fidelity(U, desc["comp_rows"], list(range(8)), T)
    assert F1 == pytest.approx(F2, rel=1e-12)


def test_idle_evolution_is_the_identity_in_the_dressed_frame():
    # drives off: U_lab = exp(-i H0 T) (dense), psi_I(T) = exp(i H_f T) U_lab v_j,
    # and M_ij = <w_i | psi_I,j(T)> = delta_ij, while the product basis shows
    # the static ZZ phases
    desc = _ring()
    o = OracleSystem(desc)
    Tt = 37.0
    V, phi, W = eb.eigenbasis_targets(o, desc["comp_rows"], np.eye(8), Tt)
    H = static_hamiltonian(o)
    f = eb.frame_diagonal(o)
    psiT = np.exp(1j * f * Tt)[:, None] * (expm(-1j * H * Tt) @ V)
    M = W.conj().T @ psiT
    assert np.abs(M - np.eye(8)).max() <= 1e-10
    assert state_fidelity(psiT, phi)[0] == pytest.approx(1.0, abs=1e-12)
    B = basis_columns(o.D, desc["comp_rows"])
    Fprod, _ = fidelity(np.exp(1j * f * Tt)[:, None] * (expm(-1j * H * Tt) @ B),
                        desc["comp_rows"], list(range(8)), np.eye(8))
    assert Fprod < 1.0 - 1e-6


def test_one_qubit_optimum_is_the_nuclear_norm():
    # von Neumann: max over unitaries a, b of |Tr(T^dag a M b)| = sum of the
    # singular values of M for a unitary T
    rng = np.random.default_rng(7)
    for _ in range(5):
        M = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        T = _haar(2, rng)
        F, a, b, tau = eb.su2_fidelity(M, T, 1)
        nuc = np.linalg.svd(M, compute_uv=False).sum()
        assert abs(tau) == pytest.approx(nuc, rel=1e-12)


def _cz(n):
    d = np.ones(2 ** n, dtype=complex)
    d[3 * 2 ** (n - 2):] = -1.0            # CZ on qubits (0, 1)
    return np.diag(d)


def _cnot(n):
    C = np.eye(4, dtype=complex)[[0, 1, 3, 2]]
    return np.kron(C, np.eye(2 ** (n - 2)))


@pytest.mark.parametrize("n,kind", [(2, "cz"), (2, "cnot"), (3, "cz"), (3, "cnot"),
                                    (3, "local")])
def test_recovers_targets_scrambled_by_local_unitaries(n, kind):
    # the gates the compensation is meant for (App. D: CNOT from a
    # cross-resonance pulse, CZ) and a product of single-qubit gates; the
    # search is local, and for generic entangling (Haar) targets it can stop
    # below the maximum
    rng = np.random.default_rng(10 + n)
    if kind == "cz":
        T = _cz(n)
    elif kind == "cnot":
        T = _cnot(n)
    else:
        T = np.ones((1, 1), dtype=complex)
        for _ in range(n):
            T = np.kron(T, _haar(2, rng))
    A = np.ones((1, 1), dtype=complex)
    B = np.ones((1, 1), dtype=complex)
    for _ in range(n):
        A = np.kron(A, _haar(2, rng))
        B = np.kron(B, _haar(2, rng))
    M = A.conj().T @ T @ B.conj().T
    F, a, b, tau = eb.su2_fidelity(M, T, n)
    assert F == pytest.approx(1.0, abs=1e-10)


def test_ordering_against_phase_only_and_plain_fidelity():
    rng = np.random.default_rng(21)
    for n in (2, 3):
        dc = 2 ** n
        T = _haar(dc, rng)
        M = 0.7 * _haar(dc, rng) + 0.2 * (rng.normal(size=(dc, dc)) + 1j * rng.normal(size=(dc, dc)))
        Fp = abs(np.trace(T.conj().T @ M)) ** 2 / dc ** 2
        Fz = zcomp_fidelity(M, T, n)[0]
        Fs = eb.su2_fidelity(M, T, n)[0]
        assert Fs >= Fz - 1e-12 and Fz >= Fp - 1e-12


def test_compensated_cotangent_is_the_plain_one_of_the_compensated_target():
    # envelope theorem: at the optimum the gates are stationary, so
    # dL_comp/dM* equals the plain cotangent with T' = A^dag T B^dag
    rng = np.random.default_rng(31)
    n, dc = 2, 4
    T = _haar(dc, rng)
    M = 0.8 * _haar(dc, rng) + 0.1 * (rng.normal(size=(dc, dc)) + 1j * rng.normal(size=(dc, dc)))
    F, a, b, tau = eb.su2_fidelity(M, T, n)
    Tp = eb.su2_target(T, a, b)
    rows = list(range(dc))
    lam = cotangent((dc, dc), rows, rows, Tp, np.trace(Tp.conj().T @ M))
    dM = rng.normal(size=(dc, dc)) + 1j * rng.normal(size=(dc, dc))
    e = 1e-6
    Lp = 1 - eb.su2_fidelity(M + e * dM, T, n)[0]
    Lm = 1 - eb.su2_fidelity(M - e * dM, T, n)[0]
    assert (Lp - Lm) / (2 * e) == pytest.approx(2 * np.vdot(lam, dM).real, rel=1e-6)
