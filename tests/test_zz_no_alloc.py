"""The allocation-free adjoint (workspace in the library's static device
array) against the adjoint with a caller workspace, through the C ABI: two
calls in a row, the second on a smaller system, each bitwise equal to the
workspace entry point's result and within the gradient bar of the oracle."""
import numpy as np
import pytest

import scp_inputs as si
from oracle.system import OracleSystem
from oracle.adjoint import loss_and_grad

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _ring(n_modes, d, T, n, seed):
    s = si.transmon_ring(si.rng_for(7, seed), n_modes, d, T, n)
    return si._finish(s, [d] * n_modes, target=si.cz_target(n_modes))


def _both(scp, desc):
    g = scp.System(desc)
    g.set_engine("register")   # the allocation-free adjoint's engine
    psi0 = scp.basis_columns(g.D, desc["columns"])
    opts = g.opts(psi0.shape[0], with_ckpt=1)
    ws = g.workspace(opts, with_grad=True)
    U = g.propagate(psi0, opts=opts, workspace=ws)
    tgt = scp.Target(desc["comp_rows"], desc["comp_cols"], desc["target"])
    cot = torch.empty_like(U)
    F, _ = scp.fidelity(U, tgt, cotangent=cot)
    ref = g.adjoint(cot, opts, ws, psi0=psi0)
    got = g.adjoint_noalloc(cot, g.opts(psi0.shape[0]), psi0)
    g.close()
    return F, ref, got


def test_noalloc_adjoint_equals_the_workspace_adjoint(scp):
    big = _ring(5, 3, T=6.0, n=300, seed=1)      # D = 243, 32 columns
    small = _ring(3, 3, T=3.0, n=120, seed=2)    # D = 27, 8 columns
    for name, desc in (("ring5", big), ("ring3", small)):
        print(f"[noalloc] {name}", flush=True)
        F, ref, got = _both(scp, desc)
        assert np.array_equal(ref, got), name
        _, Fo, _, _, go = loss_and_grad(OracleSystem(desc))
        assert abs(F - Fo) <= 1e-6
        assert np.abs(got - go).max() <= 1e-4 * np.abs(go).max()


def test_noalloc_adjoint_refuses_workloads_beyond_the_scratch(scp):
    desc = si.config5()
    g = scp.System(desc)
    opts = g.opts(len(desc["columns"]))
    psi0 = torch.zeros((1, g.D), dtype=torch.complex64, device="cuda")
    with pytest.raises(scp.ScpError, match="EINVAL.*static scratch"):
        g.adjoint_noalloc(psi0, opts, psi0)
    g.close()
