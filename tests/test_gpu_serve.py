"""Serving (continuous batching) on the GPU: results equal the direct path
and the oracle, do not depend on the mix, and admission respects the HBM
budget."""
import copy

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
    from paper_2406_18155_amd import serve
    m.serve = serve
    return m


def short_request(r, T=4.0):
    """Serving request r with its pulse shortened to T ns (50 steps/ns)."""
    q = si.serving_request(r)
    scale = T / q["T"]
    q["T"] = T
    q["n_steps"] = int(round(50 * T))
    for dr in q["drives"]:
        dr["sigma"] *= scale
    return q


def direct(scp, desc, want_grad, engine="auto"):
    """The same solve through scp_propagate / scp_propagate_adjoint on the
    engine the server uses; returns F, the gradient and that engine."""
    g = scp.System(desc)
    g.set_engine(engine)
    psi0 = scp.basis_columns(g.D, desc["columns"])
    opts = g.opts(psi0.shape[0], with_ckpt=1)
    used = g.engine(opts, with_grad=True)
    ws = g.workspace(opts, with_grad=True)
    U = g.propagate(psi0, opts=opts, workspace=ws)
    cot = torch.empty_like(U)
    F, _ = scp.fidelity(U, scp.Target(desc["comp_rows"], desc["comp_cols"], desc["target"]),
                        cotangent=cot)
    grad = g.adjoint(cot, opts, ws) if want_grad else None
    g.close()
    return F, grad, used


@pytest.mark.parametrize("engine", ["register", "auto"])
def test_server_equals_direct_path_and_oracle(scp, engine):
    # "register": every request in the batched register-layout kernels; "auto":
    # the small devices' requests on the gather engine in chunks of their own
    reqs = [short_request(r) for r in range(6)]
    srv = scp.serve.Server(64 << 30, max_active=8, chunk_work=3e5, engine=engine)
    ids = [srv.submit(q, True) for q in reqs]
    res = scp.serve.drain(srv, ids)
    used = []
    for q, rid in zip(reqs, ids):
        r = res[rid]
        assert r["state"] == "done"
        F, g, eng = direct(scp, q, True, engine)
        used.append(eng)
        print(f"[serve] {q['family']} N={len(q['modes'])} d={q['modes'][0]['trunc']} {eng}",
              flush=True)
        assert r["F"] == F
        assert np.array_equal(r["grad"], g)
    assert ("gather" in used) == (engine == "auto")
    # two of them against the oracle
    for q, rid in list(zip(reqs, ids))[:2]:
        L, Fo, tau, U, go = loss_and_grad(OracleSystem(q))
        assert abs(res[rid]["F"] - Fo) <= 1e-6
        assert np.abs(res[rid]["grad"] - go).max() <= 1e-4 * np.abs(go).max()
    srv.close()


@pytest.mark.parametrize("engine", ["register", "auto"])
def test_result_is_the_same_alone_and_in_a_mix(scp, engine):
    target = short_request(3)
    mix = [short_request(r) for r in range(10, 22)]
    srv = scp.serve.Server(64 << 30, max_active=4, chunk_work=2e5, engine=engine)
    rid = srv.submit(target, True)
    alone = scp.serve.drain(srv, [rid])[rid]
    srv.close()
    srv = scp.serve.Server(64 << 30, max_active=16, chunk_work=5e5, engine=engine)
    ids = [srv.submit(q, q["want_grad"]) for q in mix[:6]]
    rid2 = srv.submit(target, True)
    ids += [srv.submit(q, q["want_grad"]) for q in mix[6:]]
    res = scp.serve.drain(srv, ids + [rid2])
    assert res[rid2]["state"] == "done"
    assert res[rid2]["F"] == alone["F"]
    assert np.array_equal(res[rid2]["grad"], alone["grad"])
    assert all(res[i]["state"] == "done" for i in ids)
    srv.close()


def test_admission_waits_for_memory(scp):
    reqs = [short_request(r, T=2.0) for r in range(8)]
    # budget for about two requests at a time
    sizes = [scp.serve.request_bytes(q, True) for q in reqs]
    srv = scp.serve.Server(int(2.5 * max(sizes)), max_active=64, chunk_work=2e5)
    ids = [srv.submit(q, True) for q in reqs]
    a, queued = srv.step()
    assert queued > 0 and a < len(reqs)
    res = scp.serve.drain(srv, ids)
    assert all(res[i]["state"] == "done" for i in ids)
    # admissions were staggered
    admits = sorted(res[i]["t_admit"] for i in ids)
    assert admits[-1] > admits[0]
    srv.close()


def test_request_larger_than_budget_is_refused(scp):
    q = short_request(0)
    srv = scp.serve.Server(1 << 20, max_active=4)
    with pytest.raises(scp.ScpError, match="EBUSY"):
        srv.submit(q, True)
    srv.close()
