"""GPU parity of the local continuous adjoint method (LCAM) of the product
formulas (complex FP64 on the device, reverse-time recovery of the states)
against the CPU FP64 LCAM oracle, whose gradient is pinned to central finite
differences and to reverse-mode autodiff through the product formula.

Both sides compute the same gradient in FP64 and differ in rounding order and
in the matrix exponentials (Taylor scaling and squaring on the device, Pade in
scipy on the CPU), so the bar is 1e-9 relative to the largest component."""
import numpy as np
import pytest

import scp_inputs as si
from oracle import lcam, trotter
from oracle.system import OracleSystem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _ring(n_modes, d, n_steps, seed=3, T=1.0):
    # Q4j gates are not unitary: undoing one multiplies rounding errors by up to
    # exp(|Im a| tau |h|), which the transmons' lab-frame energies make large
    # at long steps; T = 1 ns in 10 steps keeps it near 2 (the workloads' steps
    # of 0.01-0.02 ns near 1.1)
    s = si.transmon_ring(si.rng_for(9, seed), n_modes, d, T, n_steps)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


def _prefix(desc, n_steps):
    """The first n_steps steps of desc at its own step h (envelopes rescaled)."""
    import copy
    d = copy.deepcopy(desc)
    scale = n_steps / d["n_steps"]
    d["T"] *= scale
    d["n_steps"] = n_steps
    for dr in d["drives"]:
        dr["sigma"] *= scale
    return d


CASES = {
    "raw3_d3_pwc": lambda: si.random_raw_system(11, [3, 3, 3], 3, 2.0, 12, env="pwc", n_pieces=4),
    "raw3_d4_gauss": lambda: si.random_raw_system(12, [4, 4, 4], 2, 2.0, 8, env="gauss"),
    "raw2_d2": lambda: si.random_raw_system(13, [2, 2], 1, 1.5, 25, env="gauss"),
    "fluxonium3_d5": lambda: si._finish(si.fluxonium_chain(si.rng_for(2, 1), 3, 5, 1.0, 8,
                                                           n_basis_gauss=3), [5] * 3),
    "ring4_d3": lambda: _ring(4, 3, 10),
}

# every order on a raw chain with a wrap edge and on a transmon ring; the
# second-order and the complex fourth-order (non-unitary gates) elsewhere
PAIRS = [(n, o) for n in ("raw3_d3_pwc", "ring4_d3") for o in trotter.ORDERS] + \
        [(n, o) for n in ("raw3_d4_gauss", "fluxonium3_d5") for o in ("q2", "q4j")] + \
        [("raw2_d2", "q2")]


def _costate(D, S, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(D, S)) + 1j * rng.normal(size=(D, S))


def _compare(scp, desc, order, cols=None, seed=0):
    columns = desc["columns"] if cols is None else cols
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, columns, dtype=torch.complex128)
    lam = _costate(g.D, len(columns), seed)
    cot = torch.tensor(lam.T.copy(), dtype=torch.complex128, device="cuda")
    grad = g.trotter_adjoint(psi0, cot, order)
    g.close()
    o = OracleSystem(desc)
    ref = lcam.gradient(o, order, lam, np.eye(o.D)[:, columns])
    err = np.abs(grad - ref).max() / np.abs(ref).max()
    print(f"[lcam] {order} rel err {err:.2e}", flush=True)
    assert err <= TOL, err
    return grad


@pytest.mark.parametrize("name,order", PAIRS, ids=[f"{n}-{o}" for n, o in PAIRS])
def test_lcam_matches_oracle(scp, name, order):
    print(f"[lcam] {name} {order}", flush=True)
    _compare(scp, CASES[name](), order)


def test_lcam_fluxonium_chain_workload_prefix(scp):
    # the 4-fluxonium chain (d = 5, D = 625, all 16 computational columns,
    # 58 parameters) over its first 6 steps at its own step of 0.02 ns
    print("[lcam] chain4_d5 workload, 6 steps", flush=True)
    _compare(scp, _prefix(si.config3(), 6), "q2", seed=1)


@pytest.mark.parametrize("dims,n_steps,order", [([3, 3], 300, "q2"), ([2, 2, 2], 260, "q4j")],
                         ids=["raw2_d3-300-q2", "raw3_d2-260-q4j"])
def test_lcam_over_several_walk_launches(scp, dims, n_steps, order):
    # more than 128 steps: the walk runs in launches of 128 steps, each one
    # resuming from the state and costate the previous launch stored
    print(f"[lcam] raw {dims} {n_steps} steps {order}", flush=True)
    _compare(scp, si.random_raw_system(14, dims, 1, 3.0, n_steps, env="gauss"), order, seed=5)


@pytest.mark.parametrize("order", ["q2", "q4j"])
def test_lcam_single_mode_device(scp, order):
    # one driven mode, no coupling: every reduced matrix has a single fibre
    # (its sum is stored directly, not split) and no pair gate exists;
    # 140 steps take two walk launches
    print(f"[lcam] one raw mode d=4, 140 steps {order}", flush=True)
    _compare(scp, si.random_raw_system(15, [4], 1, 3.0, 140, env="gauss"), order, seed=5)


def test_lcam_full_chain_workload_against_stored_oracle(scp):
    # the whole reverse-time walk of the 4-fluxonium chain workload (5000
    # steps: 39 launches of 128 steps and a last one of 8) for 4 sampled
    # columns and a seeded costate, against the oracle's stored gradient
    # (tests/golden/make_oracle_refs.py lcam_chain)
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "lcam_chain_oracle.json")
    ref = json.load(open(path))
    desc = si.config3()
    cols = ref["columns"]
    print(f"[lcam] chain4_d5 full workload, 5000 steps, columns {cols}", flush=True)
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, cols, dtype=torch.complex128)
    lam = si.random_states(g.D, len(cols), seed=si.BASE_SEED + 88)
    cot = torch.tensor(lam.T.copy(), dtype=torch.complex128, device="cuda")
    grad = g.trotter_adjoint(psi0, cot, "q2")
    g.close()
    go = np.asarray(ref["grad"])
    err = np.abs(grad - go).max() / np.abs(go).max()
    print(f"[lcam] full chain rel err {err:.2e}", flush=True)
    assert err <= TOL, err


@pytest.mark.parametrize("order", ["q1", "q4"])
def test_lcam_single_column(scp, order):
    # one column: one workgroup per walk launch (160 steps: two launches)
    desc = si.random_raw_system(16, [3, 4], 1, 2.0, 160, env="gauss")
    print(f"[lcam] one column, raw (3, 4) padded to d = 4, {order}", flush=True)
    truncs = [m["trunc"] for m in desc["modes"]]
    g = scp.System(desc)
    col = scp.padded_indices(truncs, desc["columns"][:1])
    psi0 = scp.basis_columns(g.D, col, dtype=torch.complex128)
    o = OracleSystem(desc)
    rows = scp.padded_indices(truncs, range(o.D))
    lam = _costate(o.D, 1, 9)
    big = np.zeros((g.D, 1), dtype=np.complex128)
    big[rows, :] = lam
    cot = torch.tensor(big.T.copy(), dtype=torch.complex128, device="cuda")
    grad = g.trotter_adjoint(psi0, cot, order)
    g.close()
    ref = lcam.gradient(o, order, lam, np.eye(o.D)[:, desc["columns"][:1]])
    err = np.abs(grad - ref).max() / np.abs(ref).max()
    print(f"[lcam] one column {order} rel err {err:.2e}", flush=True)
    assert err <= TOL, err


def test_lcam_x6_workload_prefix(scp):
    # the six-fluxonium X^6 chain (d = 4, D = 4096, 148 parameters), 8 sampled
    # columns over its first 2 steps of 0.01 ns, Q4 (three pieces)
    full = si.fluxonium6_x6()
    desc = _prefix(full, 2)
    cols = [int(c) for c in np.asarray(full["columns"])[si.sampled_columns(len(full["columns"]))]]
    print("[lcam] x6 chain, 2 steps, 8 columns", flush=True)
    _compare(scp, desc, "q4", cols=cols, seed=2)


def test_lcam_is_repeatable_and_checks_its_workspace(scp):
    import ctypes as C
    from paper_2406_18155_amd._lib import SCP_EINVAL, lib
    desc = CASES["ring4_d3"]()
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    cot = torch.tensor(_costate(g.D, len(desc["columns"]), 4).T.copy(), device="cuda")
    a = g.trotter_adjoint(psi0, cot, "q4j")
    b = g.trotter_adjoint(psi0, cot, "q4j")
    assert np.array_equal(a, b)
    need = g.trotter_adjoint_workspace_bytes("q2", psi0.shape[0])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    gr = (C.c_double * g.n_params)()
    st = lib().scp_propagate_trotter_adjoint(g.handle, 1, psi0.shape[0], C.c_void_p(ws.data_ptr()),
                                             need - 1, C.c_void_p(psi0.data_ptr()),
                                             C.c_void_p(cot.data_ptr()), gr, None)
    assert st == SCP_EINVAL
    g.close()
    ring = si.config5()
    g = scp.System(ring)
    with pytest.raises(scp.ScpError, match="EINVAL.*LDS"):
        g.trotter_adjoint_workspace_bytes("q2", 256)
    g.close()


@pytest.mark.parametrize("case", ["raw3_d3_pwc-q4j", "ring4_d3-q1", "x6-q2", "raw34-q4"])
def test_lcam_from_final_state_matches_full_call(scp, case):
    # the entry that starts the walk from a given psi_I(T): bitwise the full
    # call's gradient when psi_I(T) is the product formula's own result, for
    # the split walk (small columns) and the in-place walk (the X^6 chain),
    # and over two walk launches (160 steps: only the first reads psi_I(T))
    # on a (3, 4)-truncation device; psi_I(T) is only read
    import ctypes as C
    from paper_2406_18155_amd._lib import SCP_EINVAL, lib
    name, order = case.split("-")
    if name == "x6":
        full = si.fluxonium6_x6()
        desc = _prefix(full, 2)
        cols = [int(c) for c in np.asarray(full["columns"])[si.sampled_columns(len(full["columns"]))]]
    elif name == "raw34":
        desc = si.random_raw_system(16, [3, 4], 1, 2.0, 160, env="gauss")
        cols = scp.padded_indices([3, 4], desc["columns"][:2])
    else:
        desc = CASES[name]()
        cols = desc["columns"]
    print(f"[lcam] from the final state, {name} {order}", flush=True)
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, cols, dtype=torch.complex128)
    cot = torch.tensor(_costate(g.D, len(cols), 5).T.copy(), device="cuda")
    ref = g.trotter_adjoint(psi0, cot, order)
    psiT = g.propagate_trotter(psi0, order)
    keep = psiT.clone()
    got = g.trotter_adjoint_final(psiT, cot, order)
    assert np.array_equal(got, ref)
    assert torch.equal(psiT, keep)
    need = g.trotter_adjoint_workspace_bytes(order, psi0.shape[0])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    gr = (C.c_double * g.n_params)()
    code = g.TROTTER[order]
    st = lib().scp_propagate_trotter_adjoint_final(g.handle, code, psi0.shape[0],
                                                   C.c_void_p(ws.data_ptr()), need - 1,
                                                   C.c_void_p(psiT.data_ptr()),
                                                   C.c_void_p(cot.data_ptr()), gr, None)
    assert st == SCP_EINVAL
    st = lib().scp_propagate_trotter_adjoint_final(g.handle, code, psi0.shape[0],
                                                   C.c_void_p(ws.data_ptr()), need, None,
                                                   C.c_void_p(cot.data_ptr()), gr, None)
    assert st == SCP_EINVAL
    g.close()


@pytest.mark.parametrize("name,order", [("fluxonium3_d5", "q2"), ("ring4_d3", "q4j")])
def test_lcam_through_torch_autograd(scp, name, order):
    # theta -> psi_I(T) through torch.autograd (backward: the LCAM walk from
    # the forward's result), L = sum |psi_I(T) - B|^2 in torch, whose
    # costate dL/dpsi* = psi_I(T) - B is written out for the oracle
    desc = CASES[name]()
    print(f"[lcam] autograd {name} {order}", flush=True)
    model = scp.autograd.Model(desc)
    theta = torch.tensor(model.theta0, dtype=torch.float64, requires_grad=True)
    psi0 = scp.basis_columns(model.D, desc["columns"], dtype=torch.complex128)
    B = torch.tensor(_costate(model.D, len(desc["columns"]), 7).T.copy(), device="cuda")
    U = scp.autograd.propagate_trotter(model, theta, psi0, order)
    L = ((U - B).abs() ** 2).sum()
    L.backward()
    g_auto = theta.grad.numpy()
    lam = (U.detach() - B).cpu().numpy().T
    o = OracleSystem(model.desc_at(model.theta0))
    ref = lcam.gradient(o, order, lam, np.eye(o.D)[:, desc["columns"]])
    err = np.abs(g_auto - ref).max() / np.abs(ref).max()
    print(f"[lcam] autograd {order} rel err {err:.2e}", flush=True)
    assert err <= TOL, err
    g = scp.System(model.desc_at(model.theta0))
    assert torch.equal(U.detach(), g.propagate_trotter(psi0, order))
    g.close()
