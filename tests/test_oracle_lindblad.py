"""Pins of the open-system (Lindblad) oracle against closed forms, invariants,
the closed-system oracle and finite differences.  CPU only."""
import copy
import math

import numpy as np
import pytest

import scp_inputs as si
from oracle import lindblad as lb
from oracle.fidelity import average_gate_fidelity, fidelity
from oracle.rk4 import basis_columns
from oracle.rk4 import propagate as propagate_pure
from oracle.system import OracleSystem


def raw_mode(eps, frame=None, ops=None, g1=0.0, gp=0.0):
    d = len(eps)
    z = np.zeros((d, d), dtype=np.complex128)
    m = {"kind": "raw", "EC": 0.0, "EJ": 0.0, "EL": 0.0, "ng": 0.0, "phiext": 0.0,
         "basis_dim": d, "trunc": d, "eps": np.asarray(eps, dtype=np.float64),
         "ops": ops or {"n": z, "phi": z}, "gamma1": g1, "gammaphi": gp}
    if frame is not None:
        m["frame_eps"] = np.asarray(frame, dtype=np.float64)
    return m


def idle_system(mode, T, n_steps):
    d = len(mode["eps"])
    s = {"modes": [mode], "couplings": [], "drives": [], "T": float(T), "n_steps": int(n_steps),
         "columns": list(range(d)), "comp_rows": list(range(d)),
         "comp_cols": list(range(d)), "target": np.eye(d, dtype=np.complex128)}
    return s


def run_units(desc):
    sys = OracleSystem(desc)
    st = lb.input_states(desc)
    return lb.propagate(sys, lb.matrix_units(sys.D, st)), len(st)


def test_amplitude_damping_two_level_closed_form():
    # A detuned frame gives the coherence an extra rotation: with V = diag(0, -Delta)
    # rho_01 = exp((-i Delta - gamma/2) t); populations relax as exp(-gamma t).
    g, Dl, T = 0.07, 0.9, 10.0
    desc = idle_system(raw_mode([0.0, 2.0], frame=[0.0, 2.0 + Dl], g1=g), T, 2000)
    R, dc = run_units(desc)
    e = math.exp(-g * T)
    E11 = R[1 * dc + 1]
    np.testing.assert_allclose(E11[1, 1].real, e, atol=1e-11)
    np.testing.assert_allclose(E11[0, 0].real, 1 - e, atol=1e-11)
    np.testing.assert_allclose(R[0 * dc + 1][0, 1], np.exp((-1j * Dl - g / 2) * T), atol=1e-10)
    np.testing.assert_allclose(R[0][0, 0], 1.0, atol=1e-12)   # the ground state is fixed


def test_ladder_relaxation_three_levels_closed_form():
    # Level k decays at k gamma into k-1: rho22 = e^{-2gt}, rho11 = 2 (e^{-gt} - e^{-2gt}).
    g, T = 0.05, 12.0
    desc = idle_system(raw_mode([0.0, 1.0, 2.1], g1=g), T, 2400)
    R, dc = run_units(desc)
    E22 = R[2 * dc + 2]
    a, b = math.exp(-g * T), math.exp(-2 * g * T)
    np.testing.assert_allclose([E22[2, 2].real, E22[1, 1].real, E22[0, 0].real],
                               [b, 2 * (a - b), 1 - b - 2 * (a - b)], atol=1e-11)


def test_pure_dephasing_closed_form():
    # L = sqrt(2 gphi) n: rho_ab decays as exp(-gphi (a - b)^2 t), populations fixed.
    gp, T = 0.04, 15.0
    desc = idle_system(raw_mode([0.0, 1.3, 2.4], gp=gp), T, 1500)
    R, dc = run_units(desc)
    for a in range(3):
        for b in range(3):
            np.testing.assert_allclose(R[a * dc + b][a, b], math.exp(-gp * (a - b) ** 2 * T),
                                       atol=1e-11)


def open_random(seed, dims, g1=0.03, gp=0.02, **kw):
    desc = si.random_raw_system(seed, dims, len(dims), kw.pop("T", 3.0), kw.pop("n_steps", 300),
                                **kw)
    desc["modes"] = [dict(m, gamma1=g1 * (1 + 0.3 * k), gammaphi=gp * (1 + 0.2 * k))
                     for k, m in enumerate(desc["modes"])]
    return desc


def test_trace_and_hermiticity_are_preserved():
    # tr E(E_ab) = delta_ab and E(E_ba) = E(E_ab)^dag hold exactly for every
    # Lindblad generator, so RK4 keeps them to rounding.
    desc = open_random(3, [2, 3], env="gauss")
    sys = OracleSystem(desc)
    st = list(range(sys.D))
    R = lb.propagate(sys, lb.matrix_units(sys.D, st))
    D = sys.D
    for a in range(D):
        for b in range(D):
            tr = np.trace(R[a * D + b])
            np.testing.assert_allclose(tr, 1.0 if a == b else 0.0, atol=1e-12)
            np.testing.assert_allclose(R[b * D + a], R[a * D + b].conj().T, atol=1e-13)


def test_channel_is_completely_positive():
    # Choi matrix sum_ab E_ab (x) E(E_ab) of a Lindblad channel is positive
    # semidefinite (up to the RK4 error).
    desc = open_random(4, [2, 2], g1=0.2, gp=0.1)
    sys = OracleSystem(desc)
    D = sys.D
    R = lb.propagate(sys, lb.matrix_units(D, list(range(D))))
    C = np.zeros((D * D, D * D), dtype=np.complex128)
    for a in range(D):
        for b in range(D):
            Eab = np.zeros((D, D))
            Eab[a, b] = 1.0
            C += np.kron(Eab, R[a * D + b])
    w = np.linalg.eigvalsh(0.5 * (C + C.conj().T))
    assert w.min() > -1e-9
    np.testing.assert_allclose(w.sum(), D, atol=1e-10)
    # with dissipation the channel is not unitary: the Choi rank exceeds 1
    assert np.sort(w)[-2] > 1e-4


def test_unitary_limit_matches_closed_system_oracle():
    desc = open_random(5, [2, 3], g1=0.0, gp=0.0, env="gauss", T=2.0, n_steps=800)
    sys = OracleSystem(desc)
    st = lb.input_states(desc)
    R = lb.propagate(sys, lb.matrix_units(sys.D, st))
    U = propagate_pure(sys, basis_columns(sys.D, st))
    dc = len(st)
    for a in range(dc):
        for b in range(dc):
            np.testing.assert_allclose(R[a * dc + b], np.outer(U[:, a], U[:, b].conj()),
                                       atol=1e-10)
    # average fidelity of a unitary channel: (d F + 1) / (d + 1) with F = |Tr(T^dag U)|^2/d^2
    Fp, _ = fidelity(U, desc["comp_rows"], list(range(dc)), desc["target"])
    Fa, _ = lb.average_fidelity(R, desc["comp_rows"], desc["target"])
    np.testing.assert_allclose(Fa, average_gate_fidelity(Fp, dc), atol=1e-10)


def test_average_fidelity_of_damped_and_dephased_idle_qubit():
    # Amplitude damping with sqrt(1-p) = e^{-gT/2}: entanglement fidelity
    # (1 + e^{-gT/2})^2 / 4, average fidelity (2 F_e + 1)/3; dephasing with
    # coherence factor l = e^{-gphi T}: average fidelity (2 + l)/3.
    g, gp, T = 0.05, 0.03, 8.0
    R, _ = run_units(idle_system(raw_mode([0.0, 1.0], g1=g), T, 800))
    Fa, _ = lb.average_fidelity(R, [0, 1], np.eye(2))
    Fe = (1 + math.exp(-g * T / 2)) ** 2 / 4
    np.testing.assert_allclose(Fa, (2 * Fe + 1) / 3, atol=1e-11)
    R, _ = run_units(idle_system(raw_mode([0.0, 1.0], gp=gp), T, 800))
    Fa, _ = lb.average_fidelity(R, [0, 1], np.eye(2))
    np.testing.assert_allclose(Fa, (2 + math.exp(-gp * T)) / 3, atol=1e-11)


def _loss(desc):
    sys = OracleSystem(desc)
    st = lb.input_states(desc)
    R = lb.propagate(sys, lb.matrix_units(sys.D, st))
    F, _ = lb.average_fidelity(R, desc["comp_rows"], desc["target"])
    return 1.0 - F


def _perturb(desc, idx, delta):
    d = copy.deepcopy(desc)
    i = idx
    for dr in d["drives"]:
        if i < len(dr["params"]):
            dr["params"][i] += delta
            return d
        i -= len(dr["params"])
    if i < len(d["couplings"]):
        d["couplings"][i]["g"] += delta
        return d
    i -= len(d["couplings"])
    key = "gamma1" if i % 2 == 0 else "gammaphi"
    d["modes"][i // 2][key] += delta
    return d


def test_adjoint_gradient_matches_finite_differences():
    desc = open_random(6, [2, 2], g1=0.05, gp=0.03, T=2.0, n_steps=60)
    desc["target"] = si.cz_target(2)
    sys = OracleSystem(desc)
    L, g = lb.loss_and_grad(sys)
    assert 0.0 < L < 1.0
    names = lb.param_names(sys)
    assert len(names) == len(g)
    step = 1e-6
    for i in range(len(names)):
        fd = (_loss(_perturb(desc, i, step)) - _loss(_perturb(desc, i, -step))) / (2 * step)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(fd), (names[i], fd, g[i])
