"""GPU parity of the Suzuki-Trotter product formulas (complex FP64 on the
device) against the CPU FP64 oracle of the same formulas.

Both sides are FP64 throughout and differ only in rounding order and in the
matrix exponential (Taylor scaling and squaring on the device, scipy's Pade
on the CPU), so the bar is 1e-10 in every amplitude.
"""
import numpy as np
import pytest

import scp_inputs as si
from oracle import trotter
from oracle.system import OracleSystem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _ring(n_modes, d, n_steps, seed=3):
    s = si.transmon_ring(si.rng_for(9, seed), n_modes, d, 6.0, n_steps)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


def _cols(desc, k):
    """The first k columns only (the product formula is checked column by column)."""
    return dict(desc, columns=list(desc["columns"][:k]))


def _short(desc, n_steps, T=None):
    desc = dict(desc, n_steps=n_steps)
    if T is not None:
        desc["T"] = T
    return desc


CASES = {
    # raw modes with random operators, piecewise-constant drives, chain + wrap
    "raw3_d3_pwc": lambda: si.random_raw_system(11, [3, 3, 3], 3, 2.0, 40, env="pwc", n_pieces=4),
    # raw modes, Gaussian drives with carriers, d = 4
    "raw3_d4_gauss": lambda: si.random_raw_system(12, [4, 4, 4], 2, 2.0, 30, env="gauss"),
    # two transmons, full 16 x 16 unitary
    "transmon2_d4": lambda: _short(si.config1(), 200, 4.0),
    # fluxonium chain, n(x)n and phi(x)phi couplings, d = 5
    "fluxonium3_d5": lambda: _short(si._finish(si.fluxonium_chain(si.rng_for(2, 1), 3, 5, 4.0, 60),
                                               [5] * 3), 60),
    # transmon ring of 4 (the wrap edge has its first mode after its second)
    "ring4_d3": lambda: _ring(4, 3, 80),
    # one two-level mode, no coupling (only single-mode gates)
    "rabi_d2": lambda: si.rabi_system(0.7, 0.9, 3.0, 50),
    # coupled two-level modes, D = 2048: pair gates in place with the single-mode
    # gates applied in registers beside them (d = 2)
    "raw11_d2_coupled": lambda: _cols(si.random_raw_system(15, [2] * 11, 11, 1.0, 6, env="gauss"), 8),
    # pair gates split d rows per item with D / d^2 not a multiple of 64
    "raw7_d3_split": lambda: _cols(si.random_raw_system(16, [3] * 7, 7, 1.0, 6, env="gauss"), 8),
    "raw5_d5_split": lambda: _cols(si.random_raw_system(17, [5] * 5, 5, 1.0, 6, env="gauss"), 8),
}


def _run(scp, desc, order, cols=None):
    g = scp.System(desc)
    columns = desc["columns"] if cols is None else [desc["columns"][c] for c in cols]
    psi0 = scp.basis_columns(g.D, columns, dtype=torch.complex128)
    out = g.propagate_trotter(psi0, order)
    torch.cuda.synchronize()
    return out.cpu().numpy().T, np.asarray(columns)


@pytest.mark.parametrize("order", trotter.ORDERS)
@pytest.mark.parametrize("name", list(CASES))
def test_trotter_matches_oracle(scp, name, order):
    desc = CASES[name]()
    print(f"[trotter] {name} {order}", flush=True)
    U, cols = _run(scp, desc, order)
    o = OracleSystem(desc)
    ref = trotter.propagate(o, order, psi0=np.eye(o.D)[:, cols])
    err = np.abs(U - ref).max()
    assert err <= TOL, err


def test_trotter_in_place_and_repeatable(scp):
    desc = CASES["ring4_d3"]()
    print("[trotter] in place", flush=True)
    g = scp.System(desc)
    psi = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    ref = g.propagate_trotter(psi.clone(), "q4")
    g.propagate_trotter(psi, "q4", psiT=psi)
    again = g.propagate_trotter(scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128), "q4")
    torch.cuda.synchronize()
    assert torch.equal(psi, ref) and torch.equal(again, ref)


def test_trotter_orders_and_workspace(scp):
    # Unknown orders are refused; the gate tables grow with the pieces per
    # step (Q1 and Q2 one, Q4j two, Q4 three: single-mode gates of every step,
    # piece and mode, d^2 complex FP64 each) and the passes per piece (fused
    # gates of every step, piece, pass and operation).
    print("[trotter] orders and workspace", flush=True)
    import ctypes as C
    from paper_2406_18155_amd._lib import SCP_EINVAL, lib
    desc = CASES["ring4_d3"]()
    g = scp.System(desc)
    n = C.c_size_t()
    for bad in (-1, 4, 7):
        assert lib().scp_trotter_workspace_size(g.handle, bad, C.byref(n)) == SCP_EINVAL
        assert b"order" in lib().scp_last_error()
    w = {o: g.trotter_workspace_bytes(o) for o in trotter.ORDERS}
    per_piece = desc["n_steps"] * 4 * 9 * 16
    assert per_piece <= w["q1"] < w["q2"]          # Q2 fuses two passes per step
    assert w["q4j"] - w["q2"] >= per_piece and w["q4"] - w["q4j"] >= per_piece


def _prefix(desc, n_steps):
    """The first n_steps steps of a workload at its own step dt = T / N."""
    dt = desc["T"] / desc["n_steps"]
    return dict(desc, n_steps=n_steps, T=dt * n_steps)


def test_trotter_fluxonium_chain_workload_matches_oracle(scp):
    # The 4-fluxonium chain (d = 5, D = 625, all 16 columns, steps of 0.02 ns):
    # its first 250 steps, by the symmetric second-order formula (the oracle
    # takes about 7 minutes for all 5000).
    desc = _prefix(si.config2(), 250)
    print("[trotter] fluxonium chain 4 x d5, 250 of 5000 steps, q2", flush=True)
    U, cols = _run(scp, desc, "q2")
    o = OracleSystem(desc)
    ref = trotter.propagate(o, "q2", psi0=np.eye(o.D)[:, cols])
    assert np.abs(U - ref).max() <= TOL


def test_trotter_ring8_workload_sampled_columns(scp):
    # The 8-transmon ring (d = 3, D = 6561) with all 256 columns in one
    # launch, the configuration the benchmark times: 8 sampled columns of the
    # first 150 steps against the oracle; the full 3000 steps through a
    # property that holds at any length: the 256 columns stay orthonormal
    # (every real-coefficient product formula is unitary).
    full = si.config5()
    desc = _prefix(full, 150)
    print("[trotter] ring 8 x d3, 256 columns, 150 steps, q2", flush=True)
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    out = g.propagate_trotter(psi0, "q2")
    torch.cuda.synchronize()
    pick = si.sampled_columns(len(desc["columns"]))
    U = out[pick].cpu().numpy().T
    o = OracleSystem(desc)
    cols = np.asarray(desc["columns"])[pick]
    ref = trotter.propagate(o, "q2", psi0=np.eye(o.D)[:, cols])
    assert np.abs(U - ref).max() <= TOL
    print("[trotter] ring 8 x d3, 256 columns, 3000 steps, q2 and q4", flush=True)
    g = scp.System(full)
    for order in ("q2", "q4"):
        out = g.propagate_trotter(psi0, order)
        gram = (out.conj() @ out.T).cpu().numpy()
        assert np.abs(gram - np.eye(len(full["columns"]))).max() < 1e-11, order


def test_trotter_x6_fluxonium_workload_sampled_columns(scp):
    # The shape of the paper's X^(x)6 benchmark: a 6-fluxonium multipath chain
    # at d = 4 (D = 4096, 64 columns, steps of 0.01 ns).  Its pair gates run
    # split by output row between two LDS buffers and its single-mode gates
    # in place: 8 sampled columns of the first 60 steps against the oracle.
    desc = _prefix(si.fluxonium6_x6(), 60)
    print("[trotter] X6 chain 6 x d4, 64 columns, 60 steps, q2 and q4", flush=True)
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    pick = si.sampled_columns(len(desc["columns"]))
    cols = np.asarray(desc["columns"])[pick]
    o = OracleSystem(desc)
    for order in ("q2", "q4"):
        out = g.propagate_trotter(psi0, order)
        torch.cuda.synchronize()
        U = out[pick].cpu().numpy().T
        ref = trotter.propagate(o, order, psi0=np.eye(o.D)[:, cols])
        assert np.abs(U - ref).max() <= TOL, order


@pytest.mark.parametrize("order", trotter.ORDERS)
def test_trotter_ring8_register_form_every_order(scp, order):
    # The ring's pair gates run in place with its single-mode gates applied in
    # registers (before the pair gate in the first pass, after it in the
    # second): every order over its first 20 steps, 4 sampled columns.
    desc = _prefix(si.config5(), 20)
    print(f"[trotter] ring 8 x d3, 256 columns, 20 steps, {order}", flush=True)
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    out = g.propagate_trotter(psi0, order)
    torch.cuda.synchronize()
    pick = si.sampled_columns(len(desc["columns"]), n_sample=4)
    U = out[pick].cpu().numpy().T
    o = OracleSystem(desc)
    ref = trotter.propagate(o, order, psi0=np.eye(o.D)[:, np.asarray(desc["columns"])[pick]])
    assert np.abs(U - ref).max() <= TOL
