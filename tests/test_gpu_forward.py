"""GPU parity of the forward path (build, applicator, fused RK4, fidelity)
against the CPU FP64 oracle, through the C ABI."""
import copy
import math

import numpy as np
import pytest

import scp_inputs as si
from oracle.system import OracleSystem
from oracle.rk4 import apply_generator as oracle_apply, basis_columns as oracle_cols, \
    propagate as oracle_propagate
from oracle.fidelity import fidelity as oracle_fidelity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# |F_gpu - F_oracle| bar for FP32 propagation
DF_TOL = 1e-6


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _short(desc, T=None, n=None):
    d = copy.deepcopy(desc)
    if T is not None:
        scale = T / d["T"]
        d["T"] = T
        for dr in d["drives"]:
            dr["sigma"] *= scale
    if n is not None:
        d["n_steps"] = n
    return d


def _ring(n_modes, d, T=5.0, n=250, seed=0):
    rng = si.rng_for(7, seed)
    s = si.transmon_ring(rng, n_modes, d, T, n)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


def _chain(n_modes, d, T=5.0, n=250, seed=0):
    rng = si.rng_for(8, seed)
    s = si.fluxonium_chain(rng, n_modes, d, T, n, n_basis_gauss=4, amp=0.03)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


BUILD_CASES = {
    "config1": lambda: si.config1(),
    "config2": lambda: si.config2(),
    "config5": lambda: si.config5(),
}


@pytest.mark.parametrize("name", list(BUILD_CASES))
def test_build_eigensolve_matches_oracle(scp, name):
    desc = BUILD_CASES[name]()
    print(f"[build] {name}", flush=True)
    g = scp.System(desc)
    o = OracleSystem(desc)
    for m in range(o.n_modes):
        gm = g.mode(m)
        om = o.modes[m]
        scale = max(1.0, np.abs(om["eps"]).max())
        assert np.abs(gm["eps"] - om["eps"]).max() <= 1e-12 * scale
        for name_op in om["ops"]:
            ref = om["ops"][name_op]
            rel = np.abs(gm[name_op] - ref).max() / max(1.0, np.abs(ref).max())
            print(f"[build] {name} mode {m} {name_op}: max rel err {rel:.1e}", flush=True)
            assert rel <= 1e-12, name_op
    np.testing.assert_allclose(g.carriers(), [dr["omega_d"] for dr in o.drives], rtol=1e-12)
    g.close()


APPLY_CASES = {
    "transmon2_d4": lambda: _short(si.config1(), n=40),
    "fluxonium4_d5": lambda: _short(si.config2(), T=2.0, n=40),
    "ring8_d3": lambda: _short(si.config5(), T=2.0, n=40),
    "ring3_d4": lambda: _ring(3, 4, n=40),
    "ring6_d3": lambda: _ring(6, 3, n=40),
    "chain3_d5": lambda: _chain(3, 5, n=40),
    "raw_d2": lambda: si.random_raw_system(3, [2, 2, 2, 2, 2], 5, 1.0, 40, env="gauss"),
}


@pytest.mark.parametrize("name", list(APPLY_CASES))
def test_apply_generator_matches_oracle(scp, name):
    desc = APPLY_CASES[name]()
    print(f"[apply] {name}", flush=True)
    g = scp.System(desc)
    o = OracleSystem(desc)
    rng = np.random.default_rng(1)
    S = 5
    y = rng.normal(size=(S, g.D)) + 1j * rng.normal(size=(S, g.D))
    yt = torch.tensor(y, dtype=torch.complex64, device="cuda")
    for step, stage in [(0, 0), (7, 1), (13, 2), (39, 3)]:
        out = g.apply_generator(step, stage, yt).cpu().numpy()
        ref = oracle_apply(o, step, stage, y.T.reshape(o.dims + [S])).reshape(g.D, S).T
        err = np.abs(out - ref).max() / np.abs(ref).max()
        assert err <= 2e-6, (step, stage, err)
    g.close()


def _gpu_propagate(scp, desc, S_cols=None, engine="register"):
    """Forward of the columns on the register-layout stepper or the gather
    engine (one workgroup per column in LDS)."""
    g = scp.System(desc)
    g.set_engine(engine)
    cols = desc["columns"] if S_cols is None else S_cols
    psi0 = scp.basis_columns(g.D, cols)
    U = g.propagate(psi0)
    torch.cuda.synchronize()
    return g, U


def _engines(scp, desc):
    """The engines that run this device: always the register-layout stepper,
    the gather engine where it has a stepper (64 <= D <= 4096)."""
    out = ["register"]
    g = scp.System(desc)
    try:
        g.set_engine("gather")
        out.append("gather")
    except scp.ScpError:
        pass
    g.close()
    return out


def _gpu_fid(scp, U, desc):
    tgt = scp.Target(desc["comp_rows"], desc["comp_cols"], desc["target"])
    F, tau = scp.fidelity(U, tgt)
    return F


PROP_CASES = {
    "config1": lambda: si.config1(),
    "config2_short": lambda: _short(si.config2(), T=20.0, n=1000),
    "ring3_d4": lambda: _ring(3, 4, T=10.0, n=500),
    "ring6_d3": lambda: _ring(6, 3, T=10.0, n=500),
    "chain3_d5": lambda: _chain(3, 5, T=10.0, n=500),
    "raw_pwc": lambda: si.random_raw_system(1, [2, 2, 2], 3, 2.0, 400, env="pwc"),
}


@pytest.mark.parametrize("name", list(PROP_CASES))
def test_propagate_matches_oracle(scp, name):
    desc = PROP_CASES[name]()
    o = OracleSystem(desc)
    Uo = oracle_propagate(o)                                   # (D, S)
    P = Uo[np.ix_(desc["comp_rows"], desc["comp_cols"])]
    u, _, vh = np.linalg.svd(P)
    d2 = dict(desc, target=u @ vh)
    for engine in _engines(scp, desc):
        print(f"[propagate] {name} engine={engine}", flush=True)
        g, U = _gpu_propagate(scp, desc, engine=engine)
        Ug = U.cpu().numpy().T.astype(np.complex128)
        assert np.abs(Ug - Uo).max() <= 2e-5, (engine, np.abs(Ug - Uo).max())
        Fg = _gpu_fid(scp, U, desc)
        Fo, _ = oracle_fidelity(Uo, desc["comp_rows"], desc["comp_cols"], desc["target"])
        assert abs(Fg - Fo) <= DF_TOL, (engine, Fg, Fo)
        # F ~ 1 case: target = the oracle's own computational block (nearest unitary)
        Fg1 = _gpu_fid(scp, U, d2)
        Fo1, _ = oracle_fidelity(Uo, desc["comp_rows"], desc["comp_cols"], d2["target"])
        assert Fo1 > 0.9
        assert abs(Fg1 - Fo1) <= DF_TOL, (engine, Fg1, Fo1)
        g.close()


def test_config2_full_near_unit_fidelity(scp):
    desc = si.config2()
    Uo = oracle_propagate(OracleSystem(desc))
    P = Uo[np.ix_(desc["comp_rows"], desc["comp_cols"])]
    u, _, vh = np.linalg.svd(P)
    for engine in _engines(scp, desc):
        print(f"[propagate] config2 full engine={engine}", flush=True)
        g, U = _gpu_propagate(scp, desc, engine=engine)
        for tgt in (desc["target"], u @ vh):
            d2 = dict(desc, target=tgt)
            Fg = _gpu_fid(scp, U, d2)
            Fo, _ = oracle_fidelity(Uo, desc["comp_rows"], desc["comp_cols"], tgt)
            assert abs(Fg - Fo) <= DF_TOL, (engine, Fg, Fo)
        g.close()


def test_longest_serving_run_keeps_fidelity_near_one(scp):
    # 10^4 steps (T = 200 ns at 50 steps/ns, the longest serving request): the
    # compensated FP32 update must keep |dF| <= 1e-6 where F ~ 1
    desc = _short(si.config1(), T=200.0, n=10000)
    print("[propagate] config1 T=200 ns, 10000 steps", flush=True)
    g, U = _gpu_propagate(scp, desc)
    Uo = oracle_propagate(OracleSystem(desc))
    P = Uo[np.ix_(desc["comp_rows"], desc["comp_cols"])]
    u, _, vh = np.linalg.svd(P)
    d2 = dict(desc, target=u @ vh)
    Fg = _gpu_fid(scp, U, d2)
    Fo, _ = oracle_fidelity(Uo, desc["comp_rows"], desc["comp_cols"], d2["target"])
    assert Fo > 0.99
    assert abs(Fg - Fo) <= DF_TOL, (Fg, Fo)
    g.close()


def test_config5_sampled_columns(scp):
    # all 256 columns on the GPU; the oracle on 8 seeded columns (|0..0>, |1..1> included)
    desc = si.config5()
    print("[propagate] config5 full, 8 sampled columns", flush=True)
    g, U = _gpu_propagate(scp, desc)
    samp = si.sampled_columns(256, 8)
    o = OracleSystem(desc)
    psi0 = oracle_cols(o.D, [desc["columns"][j] for j in samp])
    Uo = oracle_propagate(o, psi0)
    Ug = U.cpu().numpy()[samp].T.astype(np.complex128)
    err = np.abs(Ug - Uo).max()
    assert err <= 2e-5, err
    # overlap of each sampled column with the oracle's own (F ~ 1 per column)
    for j in range(len(samp)):
        ov = np.vdot(Uo[:, j], Ug[:, j])
        dev = abs(abs(ov) ** 2 / np.vdot(Uo[:, j], Uo[:, j]).real ** 2 - 1)
        print(f"[propagate] config5 sampled column {samp[j]}: |state F - 1| = {dev:.1e}", flush=True)
        assert dev <= DF_TOL
    g.close()


def test_ragged_and_single_column(scp):
    desc = _ring(4, 3, T=4.0, n=200)
    o = OracleSystem(desc)
    for cols in ([5], list(range(0, 81, 7)), list(range(81))):
        print(f"[propagate] ring4 cols={len(cols)}", flush=True)
        g = scp.System(desc)
        U = g.propagate(scp.basis_columns(g.D, cols))
        Uo = oracle_propagate(o, oracle_cols(o.D, cols))
        assert np.abs(U.cpu().numpy().T - Uo).max() <= 2e-5
        g.close()


def test_fidelity_kernel_matches_numpy(scp):
    rng = np.random.default_rng(4)
    D, S = 37, 9
    U = rng.normal(size=(D, S)) + 1j * rng.normal(size=(D, S))
    rows = [3, 5, 8, 13, 21, 34]
    cols = [0, 2, 3, 5, 7, 8]
    T = rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6))
    tgt = scp.Target(rows, cols, T)
    for dt in (torch.complex128, torch.complex64):
        Ut = torch.tensor(U.T.copy(), dtype=dt, device="cuda")
        cot = torch.empty_like(Ut)
        F, tau = scp.fidelity(Ut, tgt, cotangent=cot)
        Fo, tauo = oracle_fidelity(Ut.cpu().numpy().T.astype(np.complex128), rows, cols, T)
        assert F == pytest.approx(Fo, rel=1e-12)
        lam = np.zeros((D, S), complex)
        for i, r in enumerate(rows):
            for j, c in enumerate(cols):
                lam[r, c] = -(tauo / 36) * T[i, j]
        tol = 1e-12 if dt == torch.complex128 else 1e-6
        assert np.abs(cot.cpu().numpy().T - lam).max() <= tol * np.abs(lam).max()


def test_state_fidelity_kernel_matches_oracle(scp):
    from oracle.fidelity import state_cotangent, state_fidelity
    rng = np.random.default_rng(5)
    D, S = 1500, 7
    U = rng.normal(size=(D, S)) + 1j * rng.normal(size=(D, S))
    cols = [6, 0, 3]
    phi = rng.normal(size=(D, 3)) + 1j * rng.normal(size=(D, 3))
    tgt = scp.StateTarget(cols, phi.T)
    for dt in (torch.complex128, torch.complex64):
        Ut = torch.tensor(U.T.copy(), dtype=dt, device="cuda")
        cot = torch.full_like(Ut, 7.0)
        F, tau = scp.fidelity_states(Ut, tgt, cotangent=cot)
        Uh = Ut.cpu().numpy().T.astype(np.complex128)
        Fo, tauo = state_fidelity(Uh[:, cols], phi)
        assert F == pytest.approx(Fo, rel=1e-12)
        lam = np.zeros((D, S), complex)
        lam[:, cols] = state_cotangent(phi, tauo)
        tol = 1e-12 if dt == torch.complex128 else 1e-6
        assert np.abs(cot.cpu().numpy().T - lam).max() <= tol * np.abs(lam).max()
    bad = scp.StateTarget([0, 9], phi[:, :2].T)       # column 9 is outside the 7
    with pytest.raises(scp.ScpError, match="ENONFINITE"):
        scp.fidelity_states(torch.tensor(U.T.copy(), device="cuda"), bad)


def test_invalid_arguments_are_rejected(scp):
    desc = si.config1()
    bad = copy.deepcopy(desc)
    bad["modes"][1]["trunc"] = 9              # above the largest truncation
    with pytest.raises(scp.ScpError, match="EINVAL"):
        scp.System(bad)
    bad = copy.deepcopy(desc)
    bad["couplings"][0]["op_i"] = "phi"      # transmons have no phase operator
    with pytest.raises(scp.ScpError, match="EINVAL"):
        scp.System(bad)
