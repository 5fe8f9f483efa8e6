"""Seeded synthetic device / pulse descriptions (pure data, no physics).

This module is the only code shared by the CPU oracle, the tests, the
benchmark and the serving replay.  It draws device and pulse parameters from
seeded numpy PCG64 generators and returns plain Python dicts; it performs none
of the simulation's arithmetic (no Hamiltonians, no eigensolves, no carriers:
a drive whose ``omega_d`` is ``None`` asks the consumer to use the dressed 0-1
frequency of the driven mode, which each consumer computes on its own).

Units: energies and rates are angular frequencies in rad/ns (GHz x 2 pi),
times in ns, hbar = 1 (the paper stores every energy as value * 2 pi; Sec. 3.1,
parameter dictionaries).

Descriptor layout (all fields plain Python / numpy types)::

    system = {
      "modes":     [{"kind": "transmon"|"fluxonium"|"raw", "EC", "EJ", "EL",
                     "ng", "phiext", "basis_dim", "trunc",
                     # raw only: "eps" (d,), "ops": {"n": (d,d) complex,
                     #                                "phi": (d,d) complex}
                     }, ...],
      "couplings": [{"i", "j", "op_i", "op_j", "g"}, ...],     # + g op_i (x) op_j
      "drives":    [{"mode", "op", "env", "params", "omega_d", "phase",
                     "sigma"}, ...],   # c(t) = env(t; params) cos(omega_d t + phase)
      "T": float, "n_steps": int,
      "columns":   [int, ...],        # basis index of each propagated column
      "comp_rows": [int, ...],        # computational-subspace rows (d_c of them)
      "comp_cols": [int, ...],        # which propagated columns are computational
      "target":    (d_c, d_c) complex ndarray,
    }

Envelope kinds (``env``): "gauss" (params [A]; A exp(-(t-T/2)^2/(2 sigma^2))),
"gauss_basis" (params a_1..a_n; sum_j a_j exp(-(t-t_j)^2/(2 sigma_b^2)),
t_j=(j-1/2)T/n, sigma_b=T/n), "cos_ramp" (params [eps_d];
eps_d/2 (1-cos(2 pi t/T))), "const" (params [c]), "pwc" (params p_0..p_{n-1};
piece floor(step*n/n_steps) of the step being taken).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
BASE_SEED = 2406018155


def rng_for(k: int, offset: int = 0) -> np.random.Generator:
    """PCG64 generator for configuration ``k`` (1-based), or request ``offset``."""
    return np.random.Generator(np.random.PCG64(BASE_SEED + k + offset))


def _u(rng, lo, hi):
    return float(rng.uniform(lo, hi))


def transmon_mode(rng, d, ncut=10, ec_range=(0.2, 0.3), ratio=(40.0, 60.0)):
    ec = _u(rng, *ec_range) * TWO_PI
    ej = ec * _u(rng, *ratio)
    return {"kind": "transmon", "EC": ec, "EJ": ej, "EL": 0.0, "ng": 0.0,
            "phiext": 0.0, "basis_dim": 2 * ncut + 1, "trunc": int(d)}


def fluxonium_mode(rng, d, basis_dim=80, ej=(3.0, 5.0), ec=(0.8, 1.2), el=(0.8, 1.2)):
    EJ = _u(rng, *ej) * TWO_PI
    EC = _u(rng, *ec) * TWO_PI
    EL = _u(rng, *el) * TWO_PI
    return {"kind": "fluxonium", "EC": EC, "EJ": EJ, "EL": EL, "ng": 0.0,
            "phiext": math.pi, "basis_dim": int(basis_dim), "trunc": int(d)}


def comp_indices(dims):
    """Basis indices of the computational states (every mode at level 0 or 1),
    binary order with mode 0 most significant; index = sum_m a_m * stride_m."""
    n = len(dims)
    strides = [int(np.prod(dims[m + 1:])) for m in range(n)]
    out = []
    for bits in range(2 ** n):
        idx = 0
        for m in range(n):
            b = (bits >> (n - 1 - m)) & 1
            idx += b * strides[m]
        out.append(idx)
    return out


def cz_target(n_modes, pair=(0, 1)):
    """CZ on modes ``pair`` (tensor) identity on the rest, in the binary order
    of :func:`comp_indices`."""
    dc = 2 ** n_modes
    diag = np.ones(dc, dtype=np.complex128)
    for bits in range(dc):
        b0 = (bits >> (n_modes - 1 - pair[0])) & 1
        b1 = (bits >> (n_modes - 1 - pair[1])) & 1
        if b0 and b1:
            diag[bits] = -1.0
    return np.diag(diag)


def _finish(system, dims, full_unitary=False, target=None):
    comp = comp_indices(dims)
    D = int(np.prod(dims))
    if full_unitary:
        cols = list(range(D))
        comp_cols = comp
    else:
        cols = list(comp)
        comp_cols = list(range(len(comp)))
    system["columns"] = cols
    system["comp_rows"] = comp
    system["comp_cols"] = comp_cols
    system["target"] = (np.eye(len(comp), dtype=np.complex128) if target is None
                        else np.asarray(target, dtype=np.complex128))
    return system


def config1(seed_offset: int = 0):
    """2 capacitively coupled transmons, d=4, full 16x16 unitary, T=40 ns,
    2000 steps; Gaussian drive on mode 0's charge operator at its 0-1 carrier."""
    rng = rng_for(1, seed_offset)
    modes = [transmon_mode(rng, 4), transmon_mode(rng, 4)]
    couplings = [{"i": 0, "j": 1, "op_i": "n", "op_j": "n",
                  "g": _u(rng, 5e-3, 20e-3) * TWO_PI}]
    T = 40.0
    drives = [{"mode": 0, "op": "n", "env": "gauss",
               "params": [_u(rng, 0.01, 0.05) * TWO_PI],
               "omega_d": None, "phase": 0.0, "sigma": T / 4.0}]
    sys_ = {"modes": modes, "couplings": couplings, "drives": drives,
            "T": T, "n_steps": 2000}
    return _finish(sys_, [4, 4], full_unitary=True, target=cz_target(2))


def fluxonium_chain(rng, n_modes, d, T, n_steps, n_basis_gauss=20, g_range=(5e-3, 30e-3),
                    drive_modes=(0, 1), amp=0.01):
    modes = [fluxonium_mode(rng, d) for _ in range(n_modes)]
    couplings = []
    for e in range(n_modes - 1):
        couplings.append({"i": e, "j": e + 1, "op_i": "n", "op_j": "n",
                          "g": _u(rng, *g_range) * TWO_PI})
        couplings.append({"i": e, "j": e + 1, "op_i": "phi", "op_j": "phi",
                          "g": _u(rng, *g_range) * TWO_PI})
    drives = []
    for m in drive_modes:
        pars = [float(v) * TWO_PI for v in rng.uniform(-amp, amp, n_basis_gauss)]
        drives.append({"mode": m, "op": "phi", "env": "gauss_basis", "params": pars,
                       "omega_d": None, "phase": 0.0, "sigma": T / n_basis_gauss})
    return {"modes": modes, "couplings": couplings, "drives": drives,
            "T": float(T), "n_steps": int(n_steps)}


def config2(seed_offset: int = 0):
    """4 fluxonium chain (80 HO states, d=5, D=625), n(x)n and phi(x)phi per edge,
    2 phi-channels (20-Gaussian basis) on modes 0 and 1, T=100 ns, 5000 steps,
    16 computational columns."""
    rng = rng_for(2, seed_offset)
    s = fluxonium_chain(rng, 4, 5, 100.0, 5000)
    return _finish(s, [5] * 4, target=cz_target(4))


def config3(seed_offset: int = 0):
    """Config 2's device (same draws) with the CZ(q0,q1) x I x I target; the
    gradient is taken w.r.t. 40 pulse amplitudes, 4 E_J and 6 couplings."""
    s = config2(seed_offset)
    s["target"] = cz_target(4, (0, 1))
    return s


def fluxonium6_x6(seed_offset: int = 0, d: int = 4):
    """The shape of the paper's simultaneous X^(x)6 benchmark (Sec. 4.2): a
    6-fluxonium multipath chain (n(x)n and phi(x)phi per edge), phi drives on
    every mode, T = 50 ns in 5000 steps of 0.01 ns, the 64 computational
    columns and the X on every qubit as target.  The paper does not state the
    truncation; d = 4 gives D = 4096."""
    rng = rng_for(6, seed_offset)
    s = fluxonium_chain(rng, 6, d, 50.0, 5000, drive_modes=tuple(range(6)))
    x6 = np.zeros((64, 64), dtype=np.complex128)
    for j in range(64):
        x6[j ^ 63, j] = 1.0
    return _finish(s, [d] * 6, target=x6)


def transmon_ring(rng, n_modes, d, T, n_steps, g_range=(5e-3, 15e-3), ring=True):
    modes = [transmon_mode(rng, d) for _ in range(n_modes)]
    couplings = []
    n_edges = n_modes if (ring and n_modes >= 3) else n_modes - 1
    for e in range(n_edges):
        couplings.append({"i": e, "j": (e + 1) % n_modes, "op_i": "n", "op_j": "n",
                          "g": _u(rng, *g_range) * TWO_PI})
    drives = []
    for m in range(n_modes):
        drives.append({"mode": m, "op": "n", "env": "gauss",
                       "params": [_u(rng, 0.01, 0.05) * TWO_PI],
                       "omega_d": None, "phase": 0.0, "sigma": T / 4.0})
    return {"modes": modes, "couplings": couplings, "drives": drives,
            "T": float(T), "n_steps": int(n_steps)}


def config5(seed_offset: int = 0):
    """8 transmon ring, d=3 (D=6561), n(x)n couplings, 8 Gaussian channels,
    T=60 ns, 3000 steps, 256 computational columns."""
    rng = rng_for(5, seed_offset)
    s = transmon_ring(rng, 8, 3, 60.0, 3000)
    return _finish(s, [3] * 8, target=cz_target(8, (0, 1)))


def open_rates(rng, n_modes, t1_us=(20.0, 60.0), tphi_us=(20.0, 60.0)):
    """Per-mode relaxation and pure-dephasing rates (1/ns) from T1, T_phi in us."""
    out = []
    for _ in range(n_modes):
        t1 = _u(rng, *t1_us) * 1e3
        tp = _u(rng, *tphi_us) * 1e3
        out.append((1.0 / t1, 1.0 / tp))
    return out


def with_rates(system, rates):
    """Copy of ``system`` whose modes carry ``gamma1`` / ``gammaphi`` (1/ns)."""
    s = dict(system)
    s["modes"] = [dict(m, gamma1=float(g1), gammaphi=float(gp))
                  for m, (g1, gp) in zip(system["modes"], rates)]
    return s


def open_chain(seed_offset: int = 0, d: int = 3, n_steps: int = 5000):
    """Open-system workload: config 2's 4-fluxonium chain (n(x)n and phi(x)phi
    per edge, 2 phi-channels with 20-Gaussian envelopes, T = 100 ns) truncated
    to ``d`` levels per mode, CZ target on modes 0 and 1, each mode with
    T1, T_phi ~ U[20, 60] us.  The channel acts on the 16 computational
    states, so 256 matrix units are propagated (D^2 = d^8 each)."""
    rng = rng_for(2, seed_offset)
    s = fluxonium_chain(rng, 4, d, 100.0, n_steps)
    s = _finish(s, [d] * 4, target=cz_target(4))
    return with_rates(s, open_rates(rng_for(20, seed_offset), 4))


def open_pair(seed_offset: int = 0, d: int = 4, n_steps: int = 2000):
    """Open-system small case: config 1's two coupled transmons (d = 4, T = 40 ns,
    Gaussian drive on mode 0) with its 4 computational states as the channel
    input (16 matrix units), CZ target, T1, T_phi ~ U[20, 60] us."""
    s = config1(seed_offset)
    s = dict(s, n_steps=int(n_steps))
    s = _finish(s, [d, d], target=cz_target(2))
    return with_rates(s, open_rates(rng_for(21, seed_offset), 2))


def sampled_columns(n_cols: int, n_sample: int = 8, seed: int = BASE_SEED + 5):
    """Seeded sample of propagated-column positions, always containing the
    first (|0...0>) and the last (|1...1>) computational column."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rest = rng.choice(np.arange(1, n_cols - 1), size=n_sample - 2, replace=False)
    return sorted([0, n_cols - 1] + [int(v) for v in rest])


def random_states(D: int, S: int, seed: int = BASE_SEED + 55):
    """Seeded complex Gaussian vectors (D x S), unnormalised: the direction by
    which a state target is moved off the oracle's own final states."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=(D, S)) + 1j * rng.normal(size=(D, S))


def random_density_matrices(D: int, S: int, rank: int = 3, seed: int = BASE_SEED + 66):
    """Seeded mixed states (S, D, D): each a random convex mix of ``rank``
    normalised complex Gaussian vectors (Hermitian, positive, trace 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((S, D, D), dtype=np.complex128)
    for s in range(S):
        w = rng.uniform(0.1, 1.0, rank)
        w = w / w.sum()
        for k in range(rank):
            v = rng.normal(size=D) + 1j * rng.normal(size=D)
            v = v / np.linalg.norm(v)
            out[s] += w[k] * np.outer(v, v.conj())
    return out


def serving_request(r: int):
    """Request ``r`` of the serving stream: family uniform over {transmon chain,
    transmon ring (>= 3 modes), fluxonium chain}; 2..6 modes; d in {3,4,5}
    redrawn until d^N <= 3125; T ~ U[20,200] ns; 50 steps/ns; all 2^N
    computational columns; one Gaussian channel per mode; CZ(q0,q1) x I target;
    half the requests ask for the gradient."""
    rng = np.random.Generator(np.random.PCG64(4_000_000 + r))
    fam = int(rng.integers(0, 3))
    n_modes = int(rng.integers(2, 7))
    if fam == 1 and n_modes < 3:
        n_modes = 3
    while True:
        d = int(rng.integers(3, 6))
        if d ** n_modes <= 3125:
            break
    T = _u(rng, 20.0, 200.0)
    n_steps = int(round(50.0 * T))
    if fam == 2:
        s = fluxonium_chain(rng, n_modes, d, T, n_steps, n_basis_gauss=1,
                            drive_modes=tuple(range(n_modes)), amp=0.01)
        for dr in s["drives"]:
            dr["env"] = "gauss"
            dr["params"] = [abs(dr["params"][0])]
            dr["sigma"] = T / 4.0
    else:
        s = transmon_ring(rng, n_modes, d, T, n_steps, g_range=(5e-3, 20e-3),
                          ring=(fam == 1))
    s = _finish(s, [d] * n_modes, target=cz_target(n_modes, (0, 1)))
    s["want_grad"] = bool(rng.integers(0, 2))
    s["family"] = ["transmon_chain", "transmon_ring", "fluxonium_chain"][fam]
    return s


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 4_000_000):
    """Arrival times (s) of ``n`` requests of a Poisson process."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    return np.cumsum(gaps)


def rabi_system(delta, omega, T, n_steps):
    """Two-level raw mode: energies (0, delta), drive on sigma_x with constant
    amplitude omega and zero carrier frequency (for the Rabi closed form)."""
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    mode = {"kind": "raw", "EC": 0.0, "EJ": 0.0, "EL": 0.0, "ng": 0.0, "phiext": 0.0,
            "basis_dim": 2, "trunc": 2, "eps": np.array([0.0, float(delta)]),
            "ops": {"n": sx, "phi": sx}}
    s = {"modes": [mode], "couplings": [],
         "drives": [{"mode": 0, "op": "n", "env": "const", "params": [float(omega)],
                     "omega_d": 0.0, "phase": 0.0, "sigma": 1.0}],
         "T": float(T), "n_steps": int(n_steps)}
    s["columns"] = [0, 1]
    s["comp_rows"] = [0, 1]
    s["comp_cols"] = [0, 1]
    s["target"] = np.eye(2, dtype=np.complex128)
    return s


def random_raw_system(seed, dims, n_edges, T, n_steps, env="pwc", n_pieces=4,
                      scale=1.0):
    """Small system of raw modes with random Hermitian operators, random
    energies and random couplings (for brute-force and parity checks)."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 1000 + seed))
    modes = []
    for d in dims:
        eps = np.concatenate([[0.0], np.sort(rng.uniform(0.5, 3.0, d - 1))]) * scale
        ops = {}
        for name in ("n", "phi"):
            a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
            ops[name] = 0.25 * (a + a.conj().T)
        modes.append({"kind": "raw", "EC": 0.0, "EJ": 0.0, "EL": 0.0, "ng": 0.0,
                      "phiext": 0.0, "basis_dim": d, "trunc": d, "eps": eps,
                      "ops": ops})
    n = len(dims)
    couplings = []
    for e in range(n_edges):
        i = e % n
        j = (e + 1) % n
        if i == j:
            continue
        couplings.append({"i": i, "j": j, "op_i": ["n", "phi"][e % 2],
                          "op_j": ["phi", "n"][e % 2], "g": float(rng.uniform(0.05, 0.3))})
    drives = []
    for m in range(n):
        if env == "pwc":
            pars = [float(v) for v in rng.uniform(-0.5, 0.5, n_pieces)]
            drives.append({"mode": m, "op": "n", "env": "pwc", "params": pars,
                           "omega_d": 0.0, "phase": 0.0, "sigma": 1.0})
        else:
            drives.append({"mode": m, "op": "n", "env": env,
                           "params": [float(rng.uniform(0.1, 0.4))],
                           "omega_d": float(rng.uniform(0.5, 2.0)),
                           "phase": float(rng.uniform(0, 1)), "sigma": T / 4.0})
    s = {"modes": modes, "couplings": couplings, "drives": drives,
         "T": float(T), "n_steps": int(n_steps)}
    return _finish(s, list(dims))
