"""GPU parity of the plain complex FP64 path (precision 1, one launch per
local term) against the CPU FP64 oracle, through the C ABI.  Both run the
same discrete method in FP64, so they agree to rounding order."""
import copy

import numpy as np
import pytest

import scp_inputs as si
from oracle.system import OracleSystem
from oracle.rk4 import basis_columns as oracle_cols, propagate as oracle_propagate
from oracle.fidelity import fidelity as oracle_fidelity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# FP64 vs FP64, same steps: only the summation order differs
U_TOL = 1e-10


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
    s = si.transmon_ring(si.rng_for(7, seed), n_modes, d, T, n)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


def _chain(n_modes, d, T=5.0, n=250, seed=0):
    s = si.fluxonium_chain(si.rng_for(8, seed), n_modes, d, T, n, n_basis_gauss=4, amp=0.03)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


def _offset_frame(desc):
    """Frame energies moved off the dressed ones: the generator gains the
    diagonal term sum_m diag(eps_m - frame_m)."""
    d = copy.deepcopy(desc)
    o = OracleSystem(desc)
    for m, md in enumerate(d["modes"]):
        md["frame_eps"] = list(o.modes[m]["eps"] + 0.01 * (m + 1) * np.arange(md["trunc"]))
    for dr in d["drives"]:
        dr["omega_d"] = o.drives[d["drives"].index(dr)]["omega_d"]
    return d


CASES = {
    "config1": lambda: si.config1(),
    "config2_short": lambda: _short(si.config2(), T=10.0, n=500),
    "ring3_d4": lambda: _ring(3, 4, T=10.0, n=500),
    "chain3_d5": lambda: _chain(3, 5, T=10.0, n=500),
    "raw_pwc": lambda: si.random_raw_system(1, [2, 2, 2], 3, 2.0, 400, env="pwc"),
    "ring3_offset_frame": lambda: _offset_frame(_ring(3, 3, T=6.0, n=300)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_plain64_matches_oracle(scp, name):
    desc = CASES[name]()
    print(f"[plain64] {name}", flush=True)
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    U = g.propagate(psi0)
    torch.cuda.synchronize()
    Uo = oracle_propagate(OracleSystem(desc))
    err = np.abs(U.cpu().numpy().T - Uo).max()
    assert err <= U_TOL, err
    tgt = scp.Target(desc["comp_rows"], desc["comp_cols"], desc["target"])
    F, _ = scp.fidelity(U, tgt)
    Fo, _ = oracle_fidelity(Uo, desc["comp_rows"], desc["comp_cols"], desc["target"])
    assert abs(F - Fo) <= 1e-12, (F, Fo)
    g.close()


def test_plain64_and_fused_fp32_agree_on_config5_sample(scp):
    # the two GPU paths on 8 sampled columns of the 8-transmon ring, shortened
    desc = _short(si.config5(), T=6.0, n=300)
    samp = si.sampled_columns(256, 8)
    cols = [desc["columns"][j] for j in samp]
    print("[plain64] ring8 d3 sampled, FP64 vs FP32 fused", flush=True)
    g = scp.System(desc)
    U64 = g.propagate(scp.basis_columns(g.D, cols, dtype=torch.complex128))
    U32 = g.propagate(scp.basis_columns(g.D, cols, dtype=torch.complex64))
    Uo = oracle_propagate(OracleSystem(desc), oracle_cols(g.D, cols))
    assert np.abs(U64.cpu().numpy().T - Uo).max() <= U_TOL
    assert np.abs(U32.cpu().numpy().T.astype(np.complex128) - Uo).max() <= 2e-5
    g.close()


def test_plain64_rejects_a_missing_workspace(scp):
    import ctypes as C
    from paper_2406_18155_amd._lib import SCP_EINVAL, lib
    desc = si.config1()
    g = scp.System(desc)
    psi0 = scp.basis_columns(g.D, desc["columns"], dtype=torch.complex128)
    out = torch.empty_like(psi0)
    o = g.opts(psi0.shape[0], precision=1)
    st = lib().scp_propagate(g.handle, C.byref(o), None, C.c_void_p(psi0.data_ptr()),
                             C.c_void_p(out.data_ptr()), None)
    assert st == SCP_EINVAL
    g.close()
