"""GPU parity of the open-system path (vectorised Lindblad equation, complex
FP32 RK4 with a compensated state, one density matrix per workgroup in LDS)
against the CPU FP64 oracle.

Bars (FP32 arithmetic, FP64 oracle): every density-matrix entry within
ENTRY_TOL absolute (entries are bounded by 1 in modulus), the channel's
average gate fidelity within 1e-6, and the channel's exact invariants (trace,
Hermiticity pairing, complete positivity) within FP32 rounding at the full
5000-step workload.
"""
import json
import os

import numpy as np
import pytest

import scp_inputs as si
from oracle import lindblad as lb
from oracle.system import OracleSystem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ENTRY_TOL = 5e-6
F_TOL = 1e-6


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _raw(seed, dims, T, n_steps, g1=0.03, gp=0.02, **kw):
    desc = si.random_raw_system(seed, dims, len(dims), T, n_steps, **kw)
    desc["modes"] = [dict(m, gamma1=g1 * (1 + 0.3 * k), gammaphi=gp * (1 + 0.2 * k))
                     for k, m in enumerate(desc["modes"])]
    return desc


def _pair_strong():
    # the two coupled transmons with T1, T_phi of ~100-300 ns so that the
    # dissipators are large next to the FP32 rounding
    desc = si.open_pair()
    desc["modes"] = [dict(m, gamma1=m["gamma1"] * 300, gammaphi=m["gammaphi"] * 300)
                     for m in desc["modes"]]
    return desc


CASES = {
    # d = 3, three modes (D^2 = 729: ragged last wave), Gaussian drives with carriers
    "raw_d3x3_gauss": lambda: _raw(21, [3, 3, 3], 3.0, 300, env="gauss"),
    # d = 2, five modes (D^2 = 1024), piecewise-constant drives
    "raw_d2x5_pwc": lambda: _raw(22, [2] * 5, 2.0, 200, env="pwc"),
    # d = 5, two modes (D^2 = 625 on 640 threads)
    "raw_d5x2_pwc": lambda: _raw(23, [5, 5], 2.0, 200, env="pwc"),
    # d = 4, three modes (D^2 = 4096, four elements per thread)
    "raw_d4x3_gauss": lambda: _raw(24, [4, 4, 4], 2.0, 120, env="gauss"),
    # relaxation only / dephasing only
    "raw_d3x2_relax": lambda: _raw(25, [3, 3], 3.0, 200, gp=0.0, env="gauss"),
    "raw_d3x2_dephase": lambda: _raw(26, [3, 3], 3.0, 200, g1=0.0, env="gauss"),
}


def _gpu(scp, desc, rho0):
    g = scp.System(desc)
    x = torch.tensor(rho0, dtype=torch.complex64, device="cuda").contiguous()
    out = g.propagate_lindblad(x).cpu().numpy().astype(np.complex128)
    g.close()
    return out


@pytest.mark.parametrize("name", sorted(CASES))
def test_mixed_states_match_oracle(scp, name):
    desc = CASES[name]()
    sys_ = OracleSystem(desc)
    rho0 = si.random_density_matrices(sys_.D, 4)
    ref = lb.propagate(sys_, rho0)
    got = _gpu(scp, desc, rho0)
    err = np.abs(got - ref).max()
    print(f"{name}: D^2={sys_.D ** 2} max |d rho| = {err:.2e}")
    assert err <= ENTRY_TOL, f"{name}: max entry error {err:.3e}"


def test_channel_fidelity_and_cotangent_match_oracle(scp):
    desc = _pair_strong()
    sys_ = OracleSystem(desc)
    st = lb.input_states(desc)
    rho0 = lb.matrix_units(sys_.D, st)
    ref = lb.propagate(sys_, rho0)
    F_ref, _ = lb.average_fidelity(ref, desc["comp_rows"], desc["target"])
    g = scp.System(desc)
    x = torch.tensor(rho0, dtype=torch.complex64, device="cuda").contiguous()
    rhoT = g.propagate_lindblad(x)
    err = np.abs(rhoT.cpu().numpy() - ref).max()
    tgt = scp.ChannelTarget(desc["comp_rows"], desc["target"])
    cot = torch.empty_like(rhoT)
    F, _ = scp.fidelity_channel(rhoT, tgt, cotangent=cot)
    lam = lb.channel_cotangent(ref.shape, desc["comp_rows"], desc["target"])
    g.close()
    print(f"pair: F={F:.9f} F_oracle={F_ref:.9f} max |d rho|={err:.2e}")
    assert err <= ENTRY_TOL
    assert abs(F - F_ref) <= F_TOL
    assert 0.2 < F_ref < 0.99   # the dissipation is visible
    np.testing.assert_allclose(cot.cpu().numpy(), lam, atol=1e-8)


def test_channel_fidelity_near_one(scp):
    # idle coupled transmons with weak dissipation against the identity: F near 1,
    # where the bar of 1e-6 on F is tight relative to 1 - F
    desc = si.open_pair()
    desc = dict(desc, drives=[dict(desc["drives"][0], params=[0.0])], T=10.0, n_steps=500,
                target=np.eye(4, dtype=np.complex128))
    sys_ = OracleSystem(desc)
    st = lb.input_states(desc)
    rho0 = lb.matrix_units(sys_.D, st)
    F_ref, _ = lb.average_fidelity(lb.propagate(sys_, rho0), desc["comp_rows"], desc["target"])
    g = scp.System(desc)
    rhoT = g.propagate_lindblad(torch.tensor(rho0, dtype=torch.complex64, device="cuda"))
    F, _ = scp.fidelity_channel(rhoT, scp.ChannelTarget(desc["comp_rows"], desc["target"]))
    g.close()
    print(f"idle pair: F={F:.10f} F_oracle={F_ref:.10f}")
    assert 0.9 < F_ref < 1.0
    assert abs(F - F_ref) <= F_TOL


def test_zero_rates_reproduce_the_closed_system(scp):
    # With no dissipation the images of the matrix units are U|a><b|U^dag with
    # U from the closed-system propagation of the same library.
    desc = dict(si.open_pair(), n_steps=1000)
    desc["T"] = 20.0
    g = scp.System(desc)
    st = lb.input_states(desc)
    rho0 = torch.tensor(lb.matrix_units(g.D, st), dtype=torch.complex64, device="cuda")
    zeros = ([0.0] * g.n_modes, [0.0] * g.n_modes)
    R = g.propagate_lindblad(rho0.contiguous(), rates=zeros).cpu().numpy()
    psi0 = scp.basis_columns(g.D, st)
    U = g.propagate(psi0).cpu().numpy().T          # D x d_c
    g.close()
    dc = len(st)
    err = max(np.abs(R[a * dc + b] - np.outer(U[:, a], U[:, b].conj())).max()
              for a in range(dc) for b in range(dc))
    # both sides are FP32 paths, each within ENTRY_TOL of the FP64 result
    # (the outer product of the closed-system columns inherits their error twice)
    assert err <= 2 * ENTRY_TOL, err


def test_full_workload_sampled_and_invariants(scp):
    """The 4-fluxonium chain (d = 3, 5000 steps, 256 matrix units) in the
    launch configuration the benchmark times: four sampled units against the
    stored oracle, and the channel's exact invariants on all 256."""
    gold = json.load(open(os.path.join(GOLDEN, "lindblad_chain_oracle.json")))
    desc = si.open_chain()
    g = scp.System(desc)
    st = [desc["columns"][c] for c in desc["comp_cols"]]
    dc = len(st)
    rho0 = scp.matrix_units(g.D, st)
    rhoT = g.propagate_lindblad(rho0)
    tgt = scp.ChannelTarget(desc["comp_rows"], desc["target"])
    F, _ = scp.fidelity_channel(rhoT, tgt)
    R = rhoT.cpu().numpy().astype(np.complex128)
    g.close()
    rows = desc["comp_rows"]
    worst = 0.0
    for k, (a, b) in enumerate(gold["samples"]):
        blk = np.array(gold["block_re"][k]) + 1j * np.array(gold["block_im"][k])
        worst = max(worst, np.abs(R[a * dc + b][np.ix_(rows, rows)] - blk).max())
        ent = np.array(gold["entries_re"][k]) + 1j * np.array(gold["entries_im"][k])
        got = np.array([R[a * dc + b][i, j] for i, j in gold["entries"]])
        worst = max(worst, np.abs(got - ent).max())
    # invariants: tr E(E_ab) = delta_ab and E(E_ba) = E(E_ab)^dag (exact for
    # the RK4 map of any Lindblad generator; complete positivity is pinned on
    # the oracle, since FP32 noise of ~1e-6 per entry moves the near-zero
    # eigenvalues of the 1296 x 1296 Choi matrix by ~1e-4)
    tr = np.einsum("sii->s", R).reshape(dc, dc)
    tr_err = np.abs(tr - np.eye(dc)).max()
    herm = max(np.abs(R[b * dc + a] - R[a * dc + b].conj().T).max()
               for a in range(dc) for b in range(dc))
    # the fidelity reduction against the FP64 formula on the same matrices
    F_cpu, _ = lb.average_fidelity(R, rows, desc["target"])
    print(f"open chain: F={F:.9f} sampled max |d rho|={worst:.2e} trace {tr_err:.1e} "
          f"herm {herm:.1e}")
    assert worst <= ENTRY_TOL
    assert tr_err <= 2e-6 and herm <= 2e-6
    assert abs(F - F_cpu) <= 1e-9


def test_refusals(scp):
    from paper_2406_18155_amd._lib import ScpError
    desc = si.open_pair()
    g = scp.System(desc)
    rho0 = scp.matrix_units(g.D, [0, 1])
    with pytest.raises(ScpError, match="non-negative"):
        g.propagate_lindblad(rho0, rates=([-1.0, 0.0], [0.0, 0.0]))
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ScpError, match="workspace"):
        g.propagate_lindblad(rho0, workspace=small)
    with pytest.raises(ScpError, match="alias"):
        g.propagate_lindblad(rho0, rhoT=rho0)
    g.close()
    big = si.random_raw_system(30, [3] * 5, 5, 1.0, 10)
    g = scp.System(big)
    with pytest.raises(ScpError, match="LDS"):
        g.lindblad_workspace_bytes()
    g.close()


# ---------------------------------------------------------------------------
# gradient (discrete adjoint of the Lindblad RK4 steps)
# ---------------------------------------------------------------------------
GRAD_TOL = 1e-4   # max |g - g_oracle| / max |g_oracle|

GRAD_CASES = {
    # two-level modes, piecewise-constant drives on every mode, one coupling
    "raw_d2x2_pwc": lambda: dict(_raw(31, [2, 2], 2.0, 120, g1=0.05, gp=0.03, env="pwc"),
                                 target=si.cz_target(2)),
    # d = 3, Gaussian drives with carriers, two couplings (a ring of three)
    "raw_d3x3_gauss": lambda: dict(_raw(32, [3, 3, 3], 1.5, 90, g1=0.04, gp=0.02, env="gauss"),
                                   target=si.cz_target(3)),
    # the coupled transmons of the open-system pair workload, 400 steps
    "pair_strong": lambda: dict(_pair_strong(), n_steps=400, T=8.0),
}


@pytest.mark.parametrize("name", sorted(GRAD_CASES))
def test_channel_gradient_matches_oracle(scp, name):
    desc = GRAD_CASES[name]()
    sys_ = OracleSystem(desc)
    st = lb.input_states(desc)
    rho0 = lb.matrix_units(sys_.D, st)
    L_ref, g_ref = lb.loss_and_grad(sys_)
    g = scp.System(desc)
    x = torch.tensor(rho0, dtype=torch.complex64, device="cuda").contiguous()
    rhoT = g.propagate_lindblad(x)
    cot = torch.empty_like(rhoT)
    F, _ = scp.fidelity_channel(rhoT, scp.ChannelTarget(desc["comp_rows"], desc["target"]),
                                cotangent=cot)
    grad = g.lindblad_adjoint(x, cot)
    g.close()
    names = lb.param_names(sys_)
    assert len(grad) == len(g_ref) == len(names)
    err = np.abs(grad - g_ref).max() / np.abs(g_ref).max()
    worst = names[int(np.argmax(np.abs(grad - g_ref)))]
    print(f"{name}: L={1 - F:.6f} L_oracle={L_ref:.6f} grad rel err {err:.2e} (worst {worst})")
    assert abs((1 - F) - L_ref) <= F_TOL
    assert err <= GRAD_TOL, (err, worst)


def test_gradient_of_a_general_cotangent(scp):
    # mixed input states and a seeded cotangent (not a fidelity's): the adjoint
    # is linear in the cotangent and exact for any of them
    desc = _raw(33, [3, 3], 2.0, 100, g1=0.05, gp=0.02, env="gauss")
    sys_ = OracleSystem(desc)
    rho0 = si.random_density_matrices(sys_.D, 3, seed=si.BASE_SEED + 90)
    rng = np.random.Generator(np.random.PCG64(si.BASE_SEED + 91))
    lam = rng.normal(size=rho0.shape) + 1j * rng.normal(size=rho0.shape)
    g_ref = lb.gradient(sys_, lam, rho0)
    g = scp.System(desc)
    x = torch.tensor(rho0, dtype=torch.complex64, device="cuda").contiguous()
    c = torch.tensor(lam, dtype=torch.complex64, device="cuda").contiguous()
    grad = g.lindblad_adjoint(x, c)
    g.close()
    err = np.abs(grad - g_ref).max() / np.abs(g_ref).max()
    print(f"general cotangent: grad rel err {err:.2e}")
    assert err <= GRAD_TOL


def test_gradient_refusals(scp):
    from paper_2406_18155_amd._lib import ScpError
    desc = si.open_pair()
    g = scp.System(desc)
    x = scp.matrix_units(g.D, [0, 1])
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ScpError, match="workspace"):
        g.lindblad_adjoint(x, torch.zeros_like(x), workspace=small)
    with pytest.raises(ScpError, match="non-negative"):
        g.lindblad_adjoint(x, torch.zeros_like(x), rates=([0.0, -1.0], [0.0, 0.0]))
    g.close()


def test_workload_shape_gradient_matches_oracle(scp):
    """The open chain's shape (d = 3, four modes: 1024 threads, seven elements
    per thread) on a shortened pulse (100 steps over 2 ns), four sampled
    matrix units and a seeded cotangent on them."""
    desc = si.open_chain(n_steps=100)
    desc = dict(desc, T=2.0)
    desc["modes"] = [dict(m, gamma1=m["gamma1"] * 1000, gammaphi=m["gammaphi"] * 1000)
                     for m in desc["modes"]]
    sys_ = OracleSystem(desc)
    st = lb.input_states(desc)
    units = lb.matrix_units(sys_.D, st)
    pick = [0, 5 * len(st) + 5, 3 * len(st) + 12, 15 * len(st) + 9]
    rho0 = units[pick]
    rng = np.random.Generator(np.random.PCG64(si.BASE_SEED + 92))
    lam = rng.normal(size=rho0.shape) + 1j * rng.normal(size=rho0.shape)
    g_ref = lb.gradient(sys_, lam, rho0)
    g = scp.System(desc)
    x = torch.tensor(rho0, dtype=torch.complex64, device="cuda").contiguous()
    c = torch.tensor(lam, dtype=torch.complex64, device="cuda").contiguous()
    grad = g.lindblad_adjoint(x, c)
    g.close()
    err = np.abs(grad - g_ref).max() / np.abs(g_ref).max()
    print(f"open chain shape: {len(grad)} params, grad rel err {err:.2e}")
    assert err <= GRAD_TOL
