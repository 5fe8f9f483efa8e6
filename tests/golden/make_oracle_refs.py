"""Write stored oracle results used by the GPU tests (calls only oracle/).

    python tests/golden/make_oracle_refs.py            # config3_oracle.json
    python tests/golden/make_oracle_refs.py config5    # config5_sampled_oracle.json
    python tests/golden/make_oracle_refs.py config5_state
        # config5_state_target.npy + config5_state_oracle.json
    python tests/golden/make_oracle_refs.py lindblad_chain
        # lindblad_chain_oracle.json
    python tests/golden/make_oracle_refs.py lcam_chain
        # lcam_chain_oracle.json

config3_oracle.json: loss, fidelity and the full gradient of the config-3
workload (4-fluxonium chain, CZ(q0,q1) x I x I target, 5000 RK4 steps),
computed by the CPU FP64 oracle (several minutes of CPU time).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import scp_inputs as si  # noqa: E402
from oracle.system import OracleSystem  # noqa: E402
from oracle.adjoint import gradient, loss_and_grad, param_names  # noqa: E402
from oracle.fidelity import state_cotangent, state_fidelity  # noqa: E402
from oracle.rk4 import basis_columns, propagate  # noqa: E402


def main():
    desc = si.config3()
    sys_ = OracleSystem(desc)
    L, F, tau, U, g = loss_and_grad(sys_)
    out = {"workload": "config3: 4 fluxonium chain, d=5, T=100 ns, 5000 RK4 steps, CZ(q0,q1) x I x I",
           "generator": "tests/golden/make_oracle_refs.py (oracle only)",
           "L": L, "F": F, "tau": [tau.real, tau.imag],
           "param_names": param_names(sys_), "grad": [float(v) for v in g]}
    with open(os.path.join(HERE, "config3_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__" and len(sys.argv) == 1:
    main()


def config5_sampled():
    """Oracle F and gradient for the 8 seeded sampled columns of the 8-transmon
    ring (fidelity restricted to the sampled computational states), for two
    targets: CZ(q0,q1) restricted to them (F ~ 5e-7), and the nearest unitary
    to the oracle's own 8 x 8 computational block ("block_target"; F ~ 5e-3,
    since the sampled columns carry little weight on the sampled rows).  The
    F ~ 1 case is config5_state below."""
    desc = sampled_config5_desc()
    sys_ = OracleSystem(desc)
    L, F, tau, U, g = loss_and_grad(sys_)
    block = U[np.ix_(desc["comp_rows"], desc["comp_cols"])]
    u, _, vh = np.linalg.svd(block)
    t1 = u @ vh
    desc1 = dict(desc, target=t1)
    L1, F1, tau1, _, g1 = loss_and_grad(OracleSystem(desc1))
    out = {"workload": "config5 sampled: 8-transmon ring d=3, T=60 ns, 3000 steps, 8 sampled "
                       "computational columns, CZ(q0,q1) restricted to them",
           "generator": "tests/golden/make_oracle_refs.py (oracle only)",
           "columns": desc["columns"], "L": L, "F": F, "tau": [tau.real, tau.imag],
           "param_names": param_names(sys_), "grad": [float(v) for v in g],
           "block_re": block.real.tolist(), "block_im": block.imag.tolist(),
           "block_target": {"target_re": t1.real.tolist(), "target_im": t1.imag.tolist(),
                         "L": L1, "F": F1, "tau": [tau1.real, tau1.imag],
                         "grad": [float(v) for v in g1]}}
    with open(os.path.join(HERE, "config5_sampled_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def sampled_config5_desc():
    desc = si.config5()
    samp = si.sampled_columns(len(desc["columns"]), 8)
    full_t = desc["target"]
    desc["comp_rows"] = [desc["comp_rows"][j] for j in samp]
    desc["columns"] = [desc["columns"][j] for j in samp]
    desc["comp_cols"] = list(range(len(samp)))
    desc["target"] = full_t[np.ix_(samp, samp)]
    return desc


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "config5":
    config5_sampled()


def config5_state():
    """Composite state cost (Sec. 4.1) of the 8 seeded sampled columns of the
    8-transmon ring at F close to 1: each target state is the oracle's own
    normalised final state moved by 0.1 (relative) along a seeded random
    direction and normalised again, so F_oracle ~ 0.99 and the gradient is not
    zero.  Writes the targets (D x 8 complex128, column j for sampled column j)
    and the oracle's F, tau and gradient."""
    desc = sampled_config5_desc()
    sys_ = OracleSystem(desc)
    psi0 = basis_columns(sys_.D, desc["columns"])
    U = propagate(sys_, psi0)
    r = si.random_states(sys_.D, U.shape[1])
    phi = U / np.linalg.norm(U, axis=0)[None, :] + 0.1 * r / np.linalg.norm(r, axis=0)[None, :]
    phi = phi / np.linalg.norm(phi, axis=0)[None, :]
    F, tau = state_fidelity(U, phi)
    lam = state_cotangent(phi, tau)
    g, _ = gradient(sys_, lam, psi0)
    np.save(os.path.join(HERE, "config5_state_target.npy"), phi, allow_pickle=False)
    out = {"workload": "config5 sampled: 8-transmon ring d=3, T=60 ns, 3000 steps, 8 sampled "
                       "computational columns, composite state cost against "
                       "config5_state_target.npy (the oracle's final states moved by 0.1)",
           "generator": "tests/golden/make_oracle_refs.py config5_state (oracle only)",
           "columns": desc["columns"], "L": 1.0 - F, "F": F, "tau": [tau.real, tau.imag],
           "param_names": param_names(sys_), "grad": [float(v) for v in g]}
    with open(os.path.join(HERE, "config5_state_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "config5_state":
    config5_state()


LINDBLAD_SAMPLES = [(0, 0), (5, 5), (3, 12), (15, 9)]


def lindblad_chain():
    """Open-system workload (4-fluxonium chain truncated to d = 3, T = 100 ns,
    5000 RK4 steps, T1 and T_phi per mode): the oracle's images of four
    sampled matrix units |s_a><s_b|, each stored as its computational 16 x 16
    block plus 64 seeded entries elsewhere (about five minutes of CPU time)."""
    from oracle import lindblad as lb
    desc = si.open_chain()
    sys_ = OracleSystem(desc)
    st = lb.input_states(desc)
    rho0 = np.stack([lb.matrix_units(sys_.D, st)[a * len(st) + b] for a, b in LINDBLAD_SAMPLES])
    R = lb.propagate(sys_, rho0)
    rng = np.random.Generator(np.random.PCG64(si.BASE_SEED + 77))
    idx = rng.integers(0, sys_.D, size=(64, 2))
    rows = desc["comp_rows"]
    out = {"workload": "open chain: 4 fluxonium chain d=3, T=100 ns, 5000 RK4 steps, "
                       "T1/T_phi per mode, 4 sampled matrix units",
           "generator": "tests/golden/make_oracle_refs.py lindblad_chain (oracle only)",
           "samples": [list(p) for p in LINDBLAD_SAMPLES], "entries": idx.tolist(),
           "block_re": [R[k][np.ix_(rows, rows)].real.tolist() for k in range(len(R))],
           "block_im": [R[k][np.ix_(rows, rows)].imag.tolist() for k in range(len(R))],
           "entries_re": [[float(R[k][i, j].real) for i, j in idx] for k in range(len(R))],
           "entries_im": [[float(R[k][i, j].imag) for i, j in idx] for k in range(len(R))]}
    with open(os.path.join(HERE, "lindblad_chain_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "lindblad_chain":
    lindblad_chain()


LCAM_SAMPLE = 4   # columns of the chain workload in the stored LCAM gradient


def lcam_chain():
    """LCAM gradient (Sec. 2.5) of the Q2 product formula on the full
    4-fluxonium chain workload (d = 5, 5000 steps of 0.02 ns, 58 parameters)
    for 4 seeded sampled computational columns and a seeded random costate
    (scp_inputs.random_states): the whole reverse-time walk of the workload,
    about 20 minutes of CPU time."""
    from oracle import lcam
    desc = si.config3()
    sys_ = OracleSystem(desc)
    pos = si.sampled_columns(len(desc["columns"]), LCAM_SAMPLE)
    cols = [int(desc["columns"][k]) for k in pos]
    lam = si.random_states(sys_.D, len(cols), seed=si.BASE_SEED + 88)
    g = lcam.gradient(sys_, "q2", lam, np.eye(sys_.D)[:, cols])
    out = {"workload": "config3 shape: 4 fluxonium chain, d=5, T=100 ns, 5000 steps, Q2",
           "generator": "tests/golden/make_oracle_refs.py lcam_chain (oracle only)",
           "columns": cols, "costate": "scp_inputs.random_states(D, 4, seed=BASE_SEED + 88)",
           "grad": [float(v) for v in g]}
    with open(os.path.join(HERE, "lcam_chain_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "lcam_chain":
    lcam_chain()
