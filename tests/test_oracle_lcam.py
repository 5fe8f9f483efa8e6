"""Pins of the LCAM oracle (the reverse-time adjoint of the product
formulas, Sec. 2.5) against facts it does not compute itself: central finite
differences of the product-formula loss, and reverse-mode autodiff through
the same product formula (the paper's TAD comparison, Sec. 4.1, where the two
gradients agree to a relative error below 1e-7)."""
import math

import numpy as np
import pytest

import scp_inputs as si
from oracle import lcam, trotter
from oracle.fd import fd_gradient
from oracle.fidelity import cotangent, fidelity
from oracle.rk4 import basis_columns
from oracle.system import OracleSystem


def _loss_fn(order):
    def f(desc):
        s = OracleSystem(desc)
        U = trotter.propagate(s, order, basis_columns(s.D, desc["columns"]))
        return 1.0 - fidelity(U, desc["comp_rows"], desc["comp_cols"], desc["target"])[0]
    return f


def _lcam(desc, order):
    s = OracleSystem(desc)
    psi0 = basis_columns(s.D, desc["columns"])
    U = trotter.propagate(s, order, psi0)
    F, tau = fidelity(U, desc["comp_rows"], desc["comp_cols"], desc["target"])
    lam = cotangent(U.shape, desc["comp_rows"], desc["comp_cols"], desc["target"], tau)
    return lcam.gradient(s, order, lam, psi0)


def _fluxonium_pair():
    desc = si.config3()
    desc["modes"] = desc["modes"][:2]
    for md in desc["modes"]:
        md["trunc"] = 3
    desc["couplings"] = desc["couplings"][:2]
    desc["drives"] = desc["drives"][:2]
    for dr in desc["drives"]:
        dr["params"] = [0.2 * v for v in dr["params"][:3]]
        dr["sigma"] = 1.0
    desc["T"], desc["n_steps"] = 1.5, 12
    return si._finish(desc, [3, 3], target=si.cz_target(2))


def _transmon_ring():
    s = si.transmon_ring(si.rng_for(7, 3), 3, 3, 4.0, 10)
    return si._finish(s, [3] * 3, target=si.cz_target(3))


@pytest.mark.parametrize("make,order", [(_fluxonium_pair, "q2"), (_fluxonium_pair, "q4j"),
                                        (_transmon_ring, "q4"), (_transmon_ring, "q1")])
def test_lcam_matches_central_differences(make, order):
    desc = make()
    g = _lcam(desc, order)
    fd = fd_gradient(desc, range(len(g)), loss_fn=_loss_fn(order))
    fdv = np.array([fd[i] for i in range(len(g))])
    scale = np.abs(fdv).max()
    assert scale > 0
    assert np.abs(g - fdv).max() <= 1e-6 * scale
    big = np.abs(fdv) > 1e-3 * scale
    np.testing.assert_allclose(g[big], fdv[big], rtol=2e-6)


def test_lcam_matches_torch_autograd_through_the_product_formula():
    # Reverse-mode autodiff (torch, float64 on the CPU) through the same Q2
    # product formula written with torch.matrix_exp, for the drive amplitudes
    # and the coupling of a random two-mode system: the paper's TAD against
    # LCAM comparison, to its 1e-7 relative bar.
    torch = pytest.importorskip("torch")
    desc = si.random_raw_system(4, [2, 3], 1, 1.5, 20, env="gauss")
    s = OracleSystem(desc)
    g = _lcam(desc, "q2")
    amp = [torch.tensor(dr["params"][0], dtype=torch.float64, requires_grad=True)
           for dr in s.drives]
    gc = torch.tensor(s.couplings[0]["g"], dtype=torch.float64, requires_grad=True)
    dims = s.dims
    psi = torch.tensor(basis_columns(s.D, desc["columns"]), dtype=torch.complex128)
    psi = psi.reshape(*dims, -1)
    h = s.h

    def apply(G, modes, x):
        if len(modes) == 1:
            m = modes[0]
            out = torch.tensordot(G, x, dims=([1], [m]))
            return torch.movedim(out, 0, m)
        i, j = modes
        G4 = G.reshape(dims[i], dims[j], dims[i], dims[j])
        out = torch.tensordot(G4, x, dims=([2, 3], [i, j]))
        return torch.movedim(out, [0, 1], [i, j])

    for n in range(s.N):
        t = n * h + 0.5 * h
        gates = []
        for m in range(s.n_modes):
            H = torch.tensor(np.diag(s.modes[m]["eps"]), dtype=torch.complex128)
            for k, dr in enumerate(s.drives):
                if dr["mode"] == m:
                    env = math.exp(-((t - 0.5 * s.T) ** 2) / (2 * dr["sigma"] ** 2))
                    c = amp[k] * env * math.cos(dr["omega_d"] * t + dr["phase"])
                    H = H + c * torch.tensor(s.op(m, dr["op"]), dtype=torch.complex128)
            gates.append(((m,), torch.linalg.matrix_exp(-0.5j * h * H)))
        for e, cdesc in enumerate(s.couplings):
            A = torch.tensor(s.op(cdesc["i"], cdesc["op_i"]), dtype=torch.complex128)
            B = torch.tensor(s.op(cdesc["j"], cdesc["op_j"]), dtype=torch.complex128)
            gates.append(((cdesc["i"], cdesc["j"]),
                          torch.linalg.matrix_exp(-0.5j * h * gc * torch.kron(A, B))))
        for modes, G in gates + gates[::-1]:
            psi = apply(G, modes, psi)
    for m in range(s.n_modes):
        ph = torch.tensor(np.exp(1j * s.frame[m] * s.T), dtype=torch.complex128)
        shape = [1] * psi.dim()
        shape[m] = len(ph)
        psi = ph.reshape(shape) * psi
    U = psi.reshape(s.D, -1)
    T = torch.tensor(desc["target"], dtype=torch.complex128)
    rows, cols = desc["comp_rows"], desc["comp_cols"]
    tau = (T.conj() * U[rows][:, cols]).sum()
    L = 1 - tau.abs() ** 2 / len(rows) ** 2
    L.backward()
    npulse = sum(len(dr["params"]) for dr in s.drives)
    tad = np.array([a.grad.item() for a in amp] + [gc.grad.item()])
    mine = np.array([g[k] for k in range(npulse)] + [g[npulse + 3 * s.n_modes]])
    rel = np.abs(mine - tad) / np.abs(tad)
    assert rel.max() < 1e-7, rel


def test_lcam_keeps_only_the_final_state():
    # the backward walk recovers the initial state from the final one
    desc = _transmon_ring()
    s = OracleSystem(desc)
    psi0 = basis_columns(s.D, desc["columns"])
    from oracle.rk4 import as_tensor
    from scipy.linalg import expm
    psi = as_tensor(s, psi0)
    for n in range(s.N):
        psi = trotter.trotter_step(s, n, psi, "q2")
    dt = s.h
    for n in range(s.N - 1, -1, -1):
        terms = trotter.local_terms(s, n, n * dt + 0.5 * dt)
        seq = list(range(len(terms)))
        for ti in reversed(seq + seq[::-1]):
            modes, H = terms[ti]
            psi = trotter.apply_local(expm(0.5j * dt * H), modes, psi)
    assert np.abs(psi.reshape(s.D, -1) - psi0).max() < 1e-12
