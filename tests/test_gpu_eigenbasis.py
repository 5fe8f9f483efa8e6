"""GPU parity of the eigenbasis transform and the local-unitary compensation
of the fidelity (App. D) against the CPU FP64 oracle (oracle/eigenbasis.py),
through the C ABI."""
import numpy as np
import pytest

import scp_inputs as si
from oracle import eigenbasis as eb
from oracle.adjoint import gradient
from oracle.fidelity import state_cotangent, state_fidelity, zcomp_fidelity
from oracle.rk4 import propagate
from oracle.system import OracleSystem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DF_TOL = 1e-6
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _ring(n_modes, T=4.0, n=200, seed=3):
    s = si.transmon_ring(si.rng_for(7, seed), n_modes, 3, T, n)
    return si._finish(s, [3] * n_modes, target=si.cz_target(n_modes))


def _chain3():
    s = si.fluxonium_chain(si.rng_for(8, 1), 3, 5, 4.0, 200, n_basis_gauss=4, amp=0.03)
    return si._finish(s, [5] * 3, target=si.cz_target(3))


CASES = {"ring3_d3": lambda: _ring(3), "chain3_d5": _chain3, "ring5_d3": lambda: _ring(5)}


@pytest.mark.parametrize("name", list(CASES))
def test_eigenbasis_states_match_oracle(scp, name):
    desc = CASES[name]()
    print(f"[eigenbasis] states {name}", flush=True)
    g = scp.System(desc)
    T = desc["target"]
    psi0, phi, W, E = g.eigenbasis_states(desc["comp_rows"], T, dtype=torch.complex128)
    o = OracleSystem(desc)
    V0, phi0, W0 = eb.eigenbasis_targets(o, desc["comp_rows"], T, desc["T"])
    _, E0 = eb.dressed_states(o, desc["comp_rows"])
    assert np.abs(E - E0).max() <= 1e-10 * np.abs(E0).max()
    assert np.abs(psi0.cpu().numpy().T - V0).max() <= 1e-10
    assert np.abs(W.cpu().numpy().T - W0).max() <= 1e-9
    assert np.abs(phi.cpu().numpy().T - phi0).max() <= 1e-9
    g.close()


@pytest.mark.parametrize("name", ["ring3_d3", "chain3_d5"])
def test_eigenbasis_fidelity_and_gradient_match_oracle(scp, name):
    # the columns start in the dressed states and the fidelity is read in the
    # dressed frame (the composite state cost against phi), FP32 propagation
    desc = CASES[name]()
    print(f"[eigenbasis] fidelity and gradient {name}", flush=True)
    g = scp.System(desc)
    psi0, phi, W, E = g.eigenbasis_states(desc["comp_rows"], desc["target"])
    n = psi0.shape[0]
    opts = g.opts(n, with_ckpt=1)
    ws = g.workspace(opts, with_grad=True)
    U = g.propagate(psi0, opts=opts, workspace=ws)
    cot = torch.empty_like(U)
    F, _ = scp.fidelity_states(U, scp.StateTarget(list(range(n)), phi.cpu().numpy()),
                               cotangent=cot)
    grad = g.adjoint(cot, opts, ws)
    g.close()
    o = OracleSystem(desc)
    V0, phi0, _ = eb.eigenbasis_targets(o, desc["comp_rows"], desc["target"], desc["T"])
    Uo = propagate(o, V0)
    Fo, tau = state_fidelity(Uo, phi0)
    go, _ = gradient(o, state_cotangent(phi0, tau), V0)
    assert abs(F - Fo) <= DF_TOL, (F, Fo)
    assert np.abs(grad - go).max() <= GRAD_TOL * np.abs(go).max()


def _haar(n, rng):
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("mode", ["z", "su2"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_local_compensation_search_matches_oracle(scp, mode, n):
    # a block near a CZ / CNOT-like gate scrambled by local unitaries, placed
    # at computational rows of an FP64 U: the device gather and the host
    # search against the oracle's search on the same block
    rng = np.random.default_rng(40 + n)
    dc = 2 ** n
    T = np.eye(dc, dtype=complex)
    if n >= 2:
        T[3 * 2 ** (n - 2):, 3 * 2 ** (n - 2):] *= -1
    A = np.ones((1, 1), dtype=complex)
    B = np.ones((1, 1), dtype=complex)
    for _ in range(n):
        A = np.kron(A, _haar(2, rng))
        B = np.kron(B, _haar(2, rng))
    M = A.conj().T @ T @ B.conj().T + 0.05 * (rng.normal(size=(dc, dc)) + 1j * rng.normal(size=(dc, dc)))
    D, S = 3 * dc + 5, dc + 2
    rows = sorted(rng.choice(D, size=dc, replace=False).tolist())
    cols = list(range(1, dc + 1))
    U = np.zeros((S, D), dtype=np.complex128)
    for i, r in enumerate(rows):
        for j, c in enumerate(cols):
            U[c, r] = M[i, j]
    Ug = torch.tensor(U, device="cuda")
    F, par, blk, Tp = scp.fidelity_local(Ug, cols, T, n, mode=mode, comp_rows=rows)
    assert np.abs(blk.cpu().numpy() - M).max() <= 1e-15
    if mode == "su2":
        Fo, a, b, _ = eb.su2_fidelity(M, T, n)
        Tpo = eb.su2_target(T, a, b)
    else:
        Fo, a, c, _ = zcomp_fidelity(M, T, n)
        from oracle.fidelity import zcomp_target
        Tpo = zcomp_target(T, a, c)
    assert abs(F - Fo) <= 1e-11, (F, Fo)
    # the compensated target is unique up to a global phase
    Tg = Tp.cpu().numpy()
    ph = np.vdot(Tpo.reshape(-1), Tg.reshape(-1))
    ph /= abs(ph)
    assert np.abs(Tg - ph * Tpo).max() <= 1e-8


def test_compensated_eigenbasis_gradient_matches_oracle(scp):
    # the full App. D path: dressed initial states, eigenbasis block, SU(2)
    # compensation, and the adjoint of the compensated loss
    desc = CASES["ring3_d3"]()
    print("[eigenbasis] compensated gradient ring3_d3", flush=True)
    g = scp.System(desc)
    psi0, _, W, E = g.eigenbasis_states(desc["comp_rows"])
    n = psi0.shape[0]
    opts = g.opts(n, with_ckpt=1)
    ws = g.workspace(opts, with_grad=True)
    U = g.propagate(psi0, opts=opts, workspace=ws)
    cot = torch.empty_like(U)
    F, par, blk, Tp = scp.fidelity_local(U, list(range(n)), desc["target"], 3, mode="su2", W=W,
                                         cotangent=cot)
    grad = g.adjoint(cot, opts, ws)
    g.close()
    o = OracleSystem(desc)
    V0, _, W0 = eb.eigenbasis_targets(o, desc["comp_rows"], np.eye(n), desc["T"])
    Uo = propagate(o, V0)
    Mo = W0.conj().T @ Uo
    Fo, a, b, _ = eb.su2_fidelity(Mo, desc["target"], 3)
    assert abs(F - Fo) <= DF_TOL, (F, Fo)
    Tpo = eb.su2_target(desc["target"], a, b)
    phi = W0 @ Tpo
    _, tau = state_fidelity(Uo, phi)
    go, _ = gradient(o, state_cotangent(phi, tau), V0)
    assert np.abs(grad - go).max() <= GRAD_TOL * np.abs(go).max()
