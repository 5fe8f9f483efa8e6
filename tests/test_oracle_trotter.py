"""Pins of the Suzuki-Trotter oracle (App. A product formulas, CPU only).

Every check compares the oracle with something it does not compute itself:
the order conditions of App. A, a closed form when the local terms commute,
dense matrix exponentials of the whole static Hamiltonian, the pinned RK4
oracle at a fine step, and unitarity.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import scp_inputs as si
from oracle import trotter
from oracle.rk4 import propagate as rk4_propagate
from oracle.system import OracleSystem


def _kron_list(mats):
    out = np.ones((1, 1), dtype=np.complex128)
    for M in mats:
        out = np.kron(out, M)
    return out


def _dense(s):
    """Static H0 and the frame H_f as dense matrices, built term by term."""
    dims = s.dims
    H = np.zeros((s.D, s.D), dtype=np.complex128)
    Hf = np.zeros((s.D, s.D), dtype=np.complex128)
    for m in range(s.n_modes):
        mats = [np.eye(d) for d in dims]
        mats[m] = np.diag(s.modes[m]["eps"])
        H += _kron_list(mats)
        mats[m] = np.diag(s.frame[m])
        Hf += _kron_list(mats)
    for c in s.couplings:
        mi = [np.eye(d) for d in dims]
        mi[c["i"]] = s.op(c["i"], c["op_i"])
        mj = [np.eye(d) for d in dims]
        mj[c["j"]] = s.op(c["j"], c["op_j"])
        H += c["g"] * _kron_list(mi) @ _kron_list(mj)
    return H, Hf


@pytest.mark.parametrize("order", trotter.ORDERS)
def test_order_conditions(order):
    # App. A: the coefficients sum to one; the fourth-order formulas also
    # cancel the cubic term (sum a^3 = 0), which with symmetric Q2 pieces
    # leaves an O(dt^5) local error.
    a, sym = trotter.coefficients(order)
    assert abs(sum(a) - 1.0) < 1e-15
    if order in ("q4", "q4j"):
        assert abs(sum(complex(x) ** 3 for x in a)) < 1e-14
    assert sym == (order != "q1")
    if order == "q4j":
        p = a[0]
        assert abs(abs(p) ** 2 - 1.0 / 3.0) < 1e-15 and p.imag < 0


@pytest.mark.parametrize("order", trotter.ORDERS)
def test_commuting_terms_are_exact(order):
    # No couplings and constant drives: the single-mode terms commute and do
    # not depend on time, so every product formula is exact for any step:
    # U_I = exp(i H_f T) (x)_m expm(-i (diag eps_m + c O_m) T).
    desc = si.random_raw_system(3, [3, 3, 3], 0, 1.7, 7, env="pwc", n_pieces=1)
    frame = []
    for md in desc["modes"]:
        md["frame_eps"] = np.asarray(md["eps"]) * 0.97 + 0.01
        frame.append(md["frame_eps"])
    s = OracleSystem(desc)
    U = trotter.propagate(s, order)
    mats = []
    for m, md in enumerate(desc["modes"]):
        c = desc["drives"][m]["params"][0]
        Hm = np.diag(md["eps"]) + c * np.asarray(md["ops"]["n"])
        mats.append(np.diag(np.exp(1j * frame[m] * s.T)) @ expm(-1j * Hm * s.T))
    ref = _kron_list(mats)[:, desc["columns"]]
    np.testing.assert_allclose(U, ref, atol=1e-12)


@pytest.mark.parametrize("order,rate", [("q1", 2), ("q2", 4), ("q4", 16), ("q4j", 8)])
def test_static_convergence_order(order, rate):
    # Two-body terms with different operators on the two modes (a transposed
    # gate or a wrong mode order would not converge to this reference):
    # global error ~ dt^n against the dense exponential of H0.  Q4j as
    # printed is two symmetric pieces with p + conj(p) = 1 and
    # p^3 + conj(p)^3 = 0; by Baker-Campbell-Hausdorff their product still
    # carries |p|^2 (conj(p)^2 - p^2) dt^4 [A, B] / 2 (A the first-order and
    # B the third-order generator of Q2), which is non-zero, so its global
    # error falls like dt^3, not dt^4.
    desc = si.random_raw_system(5, [3, 3, 3], 3, 2.0, 1, env="pwc", n_pieces=1)
    desc["drives"] = []
    desc["columns"] = list(range(27))
    s0 = OracleSystem(desc)
    H, Hf = _dense(s0)
    ref = expm(1j * Hf * s0.T) @ expm(-1j * H * s0.T)
    errs = []
    for N in (16, 32, 64):
        U = trotter.propagate(OracleSystem(dict(desc, n_steps=N)), order)
        errs.append(np.linalg.norm(U - ref, 2))
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.75 * rate < e0 / e1 < 1.3 * rate, (order, errs)


@pytest.mark.parametrize("order,rate", [("q2", 4), ("q4", 16)])
def test_driven_convergence_order_against_rk4(order, rate):
    # Gaussian drives with carriers (time-dependent single-mode terms frozen
    # at each sub-product's middle).  The symmetric formulas keep their order;
    # the reference is the pinned RK4 oracle at a much finer step.
    desc = si.random_raw_system(2, [3, 3], 1, 3.0, 1, env="gauss")
    desc["columns"] = list(range(9))
    ref = rk4_propagate(OracleSystem(dict(desc, n_steps=4000)))
    errs = []
    for N in (20, 40, 80):
        U = trotter.propagate(OracleSystem(dict(desc, n_steps=N)), order)
        errs.append(np.linalg.norm(U - ref, 2))
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.75 * rate < e0 / e1 < 1.3 * rate, (order, errs)


def test_complex_fourth_order_is_second_order_for_driven_terms():
    # Both complex pieces of Q4j are frozen at the middle of the step, so
    # for a driven system its error falls like dt^2 (third order needs the
    # static case above).  This records that reading.
    desc = si.random_raw_system(2, [3, 3], 1, 3.0, 1, env="gauss")
    desc["columns"] = list(range(9))
    ref = rk4_propagate(OracleSystem(dict(desc, n_steps=4000)))
    errs = [np.linalg.norm(trotter.propagate(OracleSystem(dict(desc, n_steps=N)), "q4j") - ref, 2)
            for N in (40, 80)]
    assert 3.0 < errs[0] / errs[1] < 5.2, errs


@pytest.mark.parametrize("order", trotter.ORDERS)
def test_unitarity(order):
    # Real coefficients give a product of unitaries.  The complex ones of Q4j
    # do not: the deviation of its product from a unitary falls with the step
    # like its local error, dt^4 per step, dt^3 over the interval.
    desc = si.random_raw_system(7, [3, 3], 1, 2.0, 30, env="gauss")
    desc["columns"] = list(range(9))
    devs = []
    for N in (30, 60):
        U = trotter.propagate(OracleSystem(dict(desc, n_steps=N)), order)
        devs.append(np.linalg.norm(U.conj().T @ U - np.eye(9), 2))
    if order == "q4j":
        assert devs[1] > 1e-8 and 6.0 < devs[0] / devs[1] < 10.0, devs
    else:
        assert max(devs) < 1e-12


def test_frame_of_the_output_matches_rk4():
    # The product formula works in the lab frame and rotates into the frame
    # of the RK4 path at the end; against the RK4 oracle the difference falls
    # like dt^4, so both are in the same frame.
    desc = si.config1()
    errs = []
    for N in (4000, 8000):
        s = OracleSystem(dict(desc, n_steps=N))
        errs.append(np.linalg.norm(trotter.propagate(s, "q4") - rk4_propagate(s), 2))
    assert errs[1] < 3e-6 and 12.0 < errs[0] / errs[1] < 20.0, errs
