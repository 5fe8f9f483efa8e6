"""Python front end of libscprop: argument marshalling over the C ABI.

Every step of the computation runs in the HIP library; this module only
converts descriptor dicts (see ``scp_inputs``) into the C structs, passes
device pointers of torch tensors and the current HIP stream, and raises on
error statuses.

State convention on the Python side: a block of S columns of dimension D is
a torch tensor of shape (S, D) (row s = column s), which is exactly the
column-major D x S layout of the C ABI.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from ._lib import (ENV, MODE_KIND, OP, CouplingDesc, DriveDesc, ModeDesc, SolveOpts, SystemDesc,
                   check, lib)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def marshal(desc):
    """(SystemDesc, keep-alive list) for a descriptor dict."""
    keep = []
    modes = (ModeDesc * len(desc["modes"]))()
    for m, md in enumerate(desc["modes"]):
        M = modes[m]
        M.kind = MODE_KIND[md["kind"]]
        M.basis_dim = int(md.get("basis_dim", md["trunc"]))
        M.trunc = int(md["trunc"])
        M.EC, M.EJ, M.EL = float(md.get("EC", 0)), float(md.get("EJ", 0)), float(md.get("EL", 0))
        M.ng, M.phiext = float(md.get("ng", 0.0)), float(md.get("phiext", 0.0))
        if md.get("frame_eps") is not None:
            M.has_frame = 1
            for a, v in enumerate(np.asarray(md["frame_eps"], dtype=np.float64)[: M.trunc]):
                M.frame_eps[a] = float(v)
        if md["kind"] == "raw":
            d = M.trunc
            eps = np.ascontiguousarray(np.asarray(md["eps"], dtype=np.float64)[:d])
            ops = np.zeros((2, d, d, 2))
            for o, name in enumerate(("n", "phi")):
                a = np.asarray(md["ops"][name], dtype=np.complex128)
                ops[o, :, :, 0] = a.real
                ops[o, :, :, 1] = a.imag
            ops = np.ascontiguousarray(ops)
            keep += [eps, ops]
            M.raw_eps = eps.ctypes.data_as(C.POINTER(C.c_double))
            M.raw_ops = ops.ctypes.data_as(C.POINTER(C.c_double))
    coups = (CouplingDesc * max(1, len(desc["couplings"])))()
    for e, c in enumerate(desc["couplings"]):
        coups[e].i, coups[e].j = int(c["i"]), int(c["j"])
        coups[e].op_i, coups[e].op_j = OP[c["op_i"]], OP[c["op_j"]]
        coups[e].g = float(c["g"])
    drives = (DriveDesc * max(1, len(desc["drives"])))()
    for k, dr in enumerate(desc["drives"]):
        R = drives[k]
        R.mode, R.op, R.env = int(dr["mode"]), OP[dr["op"]], ENV[dr["env"]]
        par = np.ascontiguousarray(np.asarray(dr["params"], dtype=np.float64))
        keep.append(par)
        R.n_par = len(par)
        R.par = par.ctypes.data_as(C.POINTER(C.c_double))
        R.has_omega = 0 if dr.get("omega_d") is None else 1
        R.omega_d = 0.0 if dr.get("omega_d") is None else float(dr["omega_d"])
        R.phase = float(dr.get("phase", 0.0))
        R.sigma = float(dr.get("sigma", 1.0))
    sd = SystemDesc()
    sd.n_modes, sd.n_couplings, sd.n_drives = len(desc["modes"]), len(desc["couplings"]), \
        len(desc["drives"])
    sd.n_steps, sd.T = int(desc["n_steps"]), float(desc["T"])
    sd.modes, sd.couplings, sd.drives = modes, coups, drives
    keep += [modes, coups, drives]
    return sd, keep


class System:
    """A built system (device tables live until ``close``)."""

    def __init__(self, desc, stream=None):
        self.desc = desc
        sd, self._keep = marshal(desc)
        h = C.c_void_p()
        check(lib().scp_build_system(C.byref(sd), _stream_ptr(stream), C.byref(h)))
        self.handle = h
        D, npar, nm = C.c_int64(), C.c_int32(), C.c_int32()
        dims = (C.c_int32 * len(desc["modes"]))()
        check(lib().scp_system_info(h, C.byref(D), C.byref(npar), C.byref(nm), dims))
        self.D, self.n_params, self.n_modes = D.value, npar.value, nm.value
        # levels per mode in the library's index space (the largest truncation;
        # a mode with fewer levels is padded with inert ones)
        self.d = int(dims[0])
        self.n_steps = int(desc["n_steps"])

    # -- introspection -------------------------------------------------------
    def mode(self, m):
        d = self.d
        eps = (C.c_double * d)()
        frame = (C.c_double * d)()
        ops = (C.c_double * (2 * d * d * 2))()
        check(lib().scp_system_mode(self.handle, m, eps, frame, ops))
        o = np.frombuffer(ops, dtype=np.float64).reshape(2, d, d, 2)
        o = o[..., 0] + 1j * o[..., 1]
        return {"eps": np.array(eps[:]), "frame": np.array(frame[:]), "n": o[0].copy(),
                "phi": o[1].copy()}

    def carriers(self):
        n = max(1, len(self.desc["drives"]))
        om = (C.c_double * n)()
        check(lib().scp_system_carriers(self.handle, om))
        return np.array(om[: len(self.desc["drives"])])

    @property
    def real_frame(self):
        """True if the FP32 path applies real operators between frame rotations."""
        v = C.c_int32()
        check(lib().scp_system_frame(self.handle, C.byref(v)))
        return bool(v.value)

    def set_real_frame(self, enable):
        """Choose the real-frame (True) or the complex (False) evaluation."""
        check(lib().scp_system_set_frame(self.handle, 1 if enable else 0))

    ENGINES = {"auto": 0, "register": 1, "gather": 2}

    def set_engine(self, engine):
        """Engine of the FP32 solves: "auto" (the gather engine for few columns
        of a small device), "register" (the register-layout stepper) or
        "gather" (the gather engine wherever it runs)."""
        check(lib().scp_system_set_engine(self.handle, self.ENGINES[engine]))

    def engine(self, opts, with_grad=False):
        """"register" or "gather": the engine a solve with these opts runs on
        ("plain64" for precision 1)."""
        v = C.c_int32()
        check(lib().scp_solve_engine(self.handle, C.byref(opts), int(with_grad), C.byref(v)))
        return {0: "plain64", 1: "register", 2: "gather"}[v.value]

    def set_timing(self, enable):
        """Bracket later forward / recompute / reverse launches with HIP events."""
        check(lib().scp_system_set_timing(self.handle, 1 if enable else 0))

    def kernel_times(self):
        """{kind: (total ms, launches)} since the last read, kinds forward,
        recompute, reverse."""
        ms = (C.c_double * 3)()
        n = (C.c_int32 * 3)()
        check(lib().scp_system_kernel_times(self.handle, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(("forward", "recompute", "reverse"))}

    def eigenbasis_states(self, labels, target=None, T=None, dtype=torch.complex64,
                          stream=None):
        """(psi0 (n, D), phi (n, D) or None, W (n, D), E (n,)): the dressed
        eigenstates of the bare labels, their dressed-frame projectors and the
        eigenbasis target states for the target (App. D basis transform)."""
        n = len(labels)
        lab = (C.c_int64 * n)(*[int(k) for k in labels])
        T = self.desc["T"] if T is None else T
        prec = 0 if dtype == torch.complex64 else 1
        psi0 = torch.empty((n, self.D), dtype=dtype, device="cuda")
        W = torch.empty((n, self.D), dtype=torch.complex128, device="cuda")
        phi = None
        tgt = None
        if target is not None:
            t = np.asarray(target, dtype=np.complex128)
            tgt = np.ascontiguousarray(np.stack([t.real, t.imag], axis=-1)).reshape(-1)
            phi = torch.empty((n, self.D), dtype=torch.complex128, device="cuda")
        E = (C.c_double * n)()
        check(lib().scp_eigenbasis_states(
            self.handle, n, lab,
            None if tgt is None else tgt.ctypes.data_as(C.POINTER(C.c_double)), float(T), prec,
            _ptr(psi0), None if phi is None else _ptr(phi), _ptr(W), E, _stream_ptr(stream)))
        return psi0, phi, W, np.array(E[:])

    def energy_tensor(self, stream=None):
        """Dressed energies labelled by bare product states (D,), rad/ns."""
        E = (C.c_double * int(self.D))()
        check(lib().scp_energy_tensor(self.handle, E, _stream_ptr(stream)))
        return np.array(E[:])

    def static_zz(self, i, j, with_grad=False, stream=None):
        """Static ZZ coupling of modes (i, j) (rad/ns) and, optionally, its
        gradient in the library's parameter order."""
        z = C.c_double()
        g = (C.c_double * max(1, self.n_params))() if with_grad else None
        check(lib().scp_static_zz(self.handle, int(i), int(j), C.byref(z), g,
                                  _stream_ptr(stream)))
        return (z.value, np.array(g[: self.n_params])) if with_grad else z.value

    # -- Suzuki-Trotter product formulas (complex FP64) -------------------
    TROTTER = {"q1": 0, "q2": 1, "q4": 2, "q4j": 3}

    def trotter_workspace_bytes(self, order):
        n = C.c_size_t()
        check(lib().scp_trotter_workspace_size(self.handle, self.TROTTER[order], C.byref(n)))
        return n.value

    def propagate_trotter(self, psi0, order="q2", psiT=None, workspace=None, stream=None):
        """psi_I(T) of the columns psi0 (S, D) complex128 by a product formula
        ("q1", "q2", "q4", "q4j"), in the frame of ``propagate``."""
        assert psi0.dtype == torch.complex128 and psi0.is_contiguous() and psi0.shape[1] == self.D
        if psiT is None:
            psiT = torch.empty_like(psi0)
        if workspace is None:
            workspace = torch.empty(self.trotter_workspace_bytes(order), dtype=torch.uint8,
                                    device=psi0.device)
        check(lib().scp_propagate_trotter(self.handle, self.TROTTER[order], psi0.shape[0],
                                          _ptr(workspace), _ptr(psi0), _ptr(psiT),
                                          _stream_ptr(stream)))
        return psiT

    def trotter_adjoint_workspace_bytes(self, order, n_cols):
        n = C.c_size_t()
        check(lib().scp_trotter_adjoint_workspace_size(self.handle, self.TROTTER[order],
                                                       int(n_cols), C.byref(n)))
        return n.value

    def trotter_adjoint(self, psi0, cotangent, order="q2", workspace=None, stream=None):
        """dL/dtheta by the local continuous adjoint of the product formula for
        the costate ``cotangent`` (S, D) complex128 of psi_I(T) of the columns
        psi0 (S, D) complex128; only the final state is kept."""
        assert psi0.dtype == torch.complex128 and psi0.is_contiguous() and psi0.shape[1] == self.D
        assert cotangent.dtype == torch.complex128 and cotangent.shape == psi0.shape
        S = psi0.shape[0]
        if workspace is None:
            workspace = torch.empty(self.trotter_adjoint_workspace_bytes(order, S),
                                    dtype=torch.uint8, device=psi0.device)
        g = (C.c_double * max(1, self.n_params))()
        check(lib().scp_propagate_trotter_adjoint(self.handle, self.TROTTER[order], S,
                                                  _ptr(workspace),
                                                  workspace.numel() * workspace.element_size(),
                                                  _ptr(psi0), _ptr(cotangent.contiguous()), g,
                                                  _stream_ptr(stream)))
        return np.array(g[: self.n_params])

    def trotter_adjoint_final(self, psiT, cotangent, order="q2", workspace=None, stream=None):
        """The same gradient as ``trotter_adjoint``, started from psi_I(T)
        (S, D) complex128 as ``propagate_trotter`` returned it for the same
        order: the internal forward is skipped."""
        assert psiT.dtype == torch.complex128 and psiT.is_contiguous() and psiT.shape[1] == self.D
        assert cotangent.dtype == torch.complex128 and cotangent.shape == psiT.shape
        S = psiT.shape[0]
        if workspace is None:
            workspace = torch.empty(self.trotter_adjoint_workspace_bytes(order, S),
                                    dtype=torch.uint8, device=psiT.device)
        g = (C.c_double * max(1, self.n_params))()
        check(lib().scp_propagate_trotter_adjoint_final(self.handle, self.TROTTER[order], S,
                                                        _ptr(workspace),
                                                        workspace.numel() * workspace.element_size(),
                                                        _ptr(psiT), _ptr(cotangent.contiguous()), g,
                                                        _stream_ptr(stream)))
        return np.array(g[: self.n_params])

    # -- open systems (vectorised Lindblad equation) --------------------------
    def rates(self):
        """Per-mode (gamma1, gammaphi) of the descriptor (1/ns; absent: 0)."""
        g1 = [float(m.get("gamma1", 0.0)) for m in self.desc["modes"]]
        gp = [float(m.get("gammaphi", 0.0)) for m in self.desc["modes"]]
        return g1, gp

    def lindblad_workspace_bytes(self):
        n = C.c_size_t()
        check(lib().scp_lindblad_workspace_size(self.handle, C.byref(n)))
        return n.value

    def propagate_lindblad(self, rho0, rhoT=None, rates=None, workspace=None, stream=None):
        """rho_I(T) of the density matrices rho0 (S, D, D) complex64 under the
        Lindblad equation with per-mode (gamma1, gammaphi) ``rates`` (default:
        the descriptor's)."""
        assert rho0.dtype == torch.complex64 and rho0.is_contiguous()
        assert rho0.shape[1:] == (self.D, self.D)
        if rhoT is None:
            rhoT = torch.empty_like(rho0)
        if workspace is None:
            workspace = torch.empty(self.lindblad_workspace_bytes(), dtype=torch.uint8,
                                    device=rho0.device)
        g1, gp = self.rates() if rates is None else rates
        n = self.n_modes
        a1 = (C.c_double * n)(*[float(v) for v in g1])
        ap = (C.c_double * n)(*[float(v) for v in gp])
        check(lib().scp_propagate_lindblad(self.handle, a1, ap, rho0.shape[0], _ptr(workspace),
                                           workspace.numel() * workspace.element_size(),
                                           _ptr(rho0), _ptr(rhoT), _stream_ptr(stream)))
        return rhoT

    def lindblad_adjoint_workspace_bytes(self, n_cols):
        n = C.c_size_t()
        check(lib().scp_lindblad_adjoint_workspace_size(self.handle, int(n_cols), C.byref(n)))
        return n.value

    def lindblad_adjoint(self, rho0, cotangent, rates=None, workspace=None, stream=None):
        """dLoss/dtheta (drive parameters, couplings, then (gamma1, gammaphi)
        per mode) for the cotangent (S, D, D) complex64 of rho_I(T) of rho0."""
        assert rho0.dtype == torch.complex64 and rho0.is_contiguous()
        assert cotangent.dtype == torch.complex64 and cotangent.shape == rho0.shape
        S = rho0.shape[0]
        if workspace is None:
            workspace = torch.empty(self.lindblad_adjoint_workspace_bytes(S), dtype=torch.uint8,
                                    device=rho0.device)
        g1, gp = self.rates() if rates is None else rates
        n = self.n_modes
        a1 = (C.c_double * n)(*[float(v) for v in g1])
        ap = (C.c_double * n)(*[float(v) for v in gp])
        npar = self.n_params - 3 * n + 2 * n     # pulse + couplings + 2 rates per mode
        g = (C.c_double * max(1, npar))()
        check(lib().scp_lindblad_adjoint(self.handle, a1, ap, S, _ptr(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _ptr(rho0), _ptr(cotangent.contiguous()), g,
                                         _stream_ptr(stream)))
        return np.array(g[:npar])

    def opts(self, n_cols, precision=0, ckpt_every=0, with_ckpt=0):
        o = SolveOpts()
        o.n_cols, o.precision, o.ckpt_every, o.with_ckpt = int(n_cols), int(precision), \
            int(ckpt_every), int(with_ckpt)
        return o

    def workspace_bytes(self, opts, with_grad=False):
        n = C.c_size_t()
        check(lib().scp_workspace_size(self.handle, C.byref(opts), int(with_grad), C.byref(n)))
        return n.value

    def workspace(self, opts, with_grad=False, device="cuda"):
        return torch.empty(self.workspace_bytes(opts, with_grad), dtype=torch.uint8, device=device)

    # -- compute ---------------------------------------------------------------
    def apply_generator(self, step, stage, y, out=None, stream=None):
        """V(t) y (FP32) at the stage time of (step, stage); y is (S, D) complex64."""
        assert y.dtype == torch.complex64 and y.is_contiguous() and y.shape[1] == self.D
        if out is None:
            out = torch.empty_like(y)
        check(lib().scp_apply_generator(self.handle, step, stage, _ptr(y), _ptr(out), y.shape[0],
                                        _stream_ptr(stream)))
        return out

    def propagate(self, psi0, psiT=None, opts=None, workspace=None, stream=None):
        prec = 0 if psi0.dtype == torch.complex64 else 1
        assert psi0.is_contiguous() and psi0.shape[1] == self.D
        if opts is None:
            opts = self.opts(psi0.shape[0], precision=prec)
        if opts.precision != prec:
            raise ValueError(f"opts.precision={opts.precision} but psi0 is {psi0.dtype}")
        if psiT is None:
            psiT = torch.empty_like(psi0)
        if workspace is None:
            workspace = self.workspace(opts, device=psi0.device)
        opts.workspace_bytes = workspace.numel() * workspace.element_size()
        check(lib().scp_propagate(self.handle, C.byref(opts), _ptr(workspace), _ptr(psi0),
                                  _ptr(psiT), _stream_ptr(stream)))
        return psiT

    def adjoint(self, cotangent, opts, workspace, psi0=None, stream=None):
        """dL/dtheta for the costate ``cotangent`` (S, D) complex64 of the final
        state.  psi0 None: the checkpoints of the preceding ``propagate`` with
        with_ckpt=1 on ``workspace``; else they are first recomputed from psi0."""
        g = (C.c_double * max(1, self.n_params))()
        opts.workspace_bytes = workspace.numel() * workspace.element_size()
        check(lib().scp_propagate_adjoint(self.handle, C.byref(opts), _ptr(workspace),
                                          None if psi0 is None else _ptr(psi0),
                                          _ptr(cotangent), g, _stream_ptr(stream)))
        return np.array(g[: self.n_params])

    def adjoint_noalloc(self, cotangent, opts, psi0, stream=None):
        """The gradient of ``adjoint(cotangent, opts, ws, psi0)`` with the
        workspace in the library's static 64 MiB device array (no device
        allocation; calls that overlap on one GPU race)."""
        g = (C.c_double * max(1, self.n_params))()
        check(lib().scp_propagate_adjoint_noalloc(self.handle, C.byref(opts), _ptr(psi0),
                                                  _ptr(cotangent), g, _stream_ptr(stream)))
        return np.array(g[: self.n_params])

    def close(self):
        if getattr(self, "handle", None):
            lib().scp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Target:
    """Device-resident fidelity inputs: computational rows/cols and target."""

    def __init__(self, comp_rows, comp_cols, target, device="cuda"):
        self.dc = len(comp_rows)
        self.rows = torch.tensor(list(comp_rows), dtype=torch.int64, device=device)
        self.cols = torch.tensor(list(comp_cols), dtype=torch.int32, device=device)
        self.target = torch.tensor(np.asarray(target, dtype=np.complex128), device=device).contiguous()
        self.tau = torch.zeros(1, dtype=torch.complex128, device=device)


def fidelity(U, tgt: Target, cotangent=None, stream=None, sync=True):
    """F = |tau|^2 / d_c^2 of U (S, D); fills ``cotangent`` (same shape) if given."""
    prec = 0 if U.dtype == torch.complex64 else 1
    S, D = U.shape
    F = C.c_double()
    check(lib().scp_fidelity(_ptr(U), D, S, prec, tgt.dc, _ptr(tgt.rows), _ptr(tgt.cols),
                             _ptr(tgt.target), _ptr(tgt.tau),
                             None if cotangent is None else _ptr(cotangent),
                             C.byref(F) if sync else None, _stream_ptr(stream)))
    return (F.value if sync else None), tgt.tau


class StateTarget:
    """Device-resident inputs of the composite state cost: the propagated
    columns it covers and their full target states (n_t, D)."""

    def __init__(self, cols, targets, device="cuda"):
        targets = np.asarray(targets, dtype=np.complex128)
        self.n_t = len(cols)
        assert targets.shape[0] == self.n_t
        self.cols = torch.tensor(list(cols), dtype=torch.int32, device=device)
        self.targets = torch.tensor(targets, device=device).contiguous()
        self.tau = torch.zeros(1, dtype=torch.complex128, device=device)


def fidelity_states(U, tgt: StateTarget, cotangent=None, stream=None, sync=True):
    """F = |sum_j <phi_j|U[cols[j]]>|^2 / n_t^2 of U (S, D) against full target
    states; fills ``cotangent`` (same shape as U) if given."""
    prec = 0 if U.dtype == torch.complex64 else 1
    S, D = U.shape
    assert tgt.targets.shape[1] == D
    F = C.c_double()
    check(lib().scp_fidelity_states(_ptr(U), D, S, prec, tgt.n_t, _ptr(tgt.cols),
                                    _ptr(tgt.targets), _ptr(tgt.tau),
                                    None if cotangent is None else _ptr(cotangent),
                                    C.byref(F) if sync else None, _stream_ptr(stream)))
    return (F.value if sync else None), tgt.tau


class ChannelTarget:
    """Device-resident inputs of the channel fidelity: the computational rows
    and the target (d_c x d_c)."""

    def __init__(self, comp_rows, target, device="cuda"):
        self.dc = len(comp_rows)
        self.rows = torch.tensor(list(comp_rows), dtype=torch.int64, device=device)
        self.target = torch.tensor(np.asarray(target, dtype=np.complex128), device=device).contiguous()
        self.ov = torch.zeros(1, dtype=torch.complex128, device=device)


def matrix_units(D, states, dtype=torch.complex64, device="cuda"):
    """The d_c^2 input matrices |s_a><s_b| (order a d_c + b), (d_c^2, D, D)."""
    dc = len(states)
    out = torch.zeros(dc * dc, D, D, dtype=dtype, device=device)
    for a in range(dc):
        for b in range(dc):
            out[a * dc + b, states[a], states[b]] = 1.0
    return out


def fidelity_channel(rhoT, tgt: ChannelTarget, cotangent=None, stream=None, sync=True):
    """Average gate fidelity (Re ov + d_c) / (d_c (d_c + 1)) of the channel whose
    matrix-unit images are rhoT (d_c^2, D, D); fills ``cotangent`` if given."""
    assert rhoT.dtype == torch.complex64 and rhoT.is_contiguous()
    S, D, D2 = rhoT.shape
    assert D == D2 and S == tgt.dc * tgt.dc
    F = C.c_double()
    check(lib().scp_fidelity_channel(_ptr(rhoT), D, tgt.dc, _ptr(tgt.rows), _ptr(tgt.target),
                                     _ptr(tgt.ov), None if cotangent is None else _ptr(cotangent),
                                     C.byref(F) if sync else None, _stream_ptr(stream)))
    return (F.value if sync else None), tgt.ov


def fidelity_local(U, cols, target, n_qubits, mode="su2", W=None, comp_rows=None,
                   cotangent=None, stream=None):
    """Fidelity with error-free single-qubit gates before and after the gate
    (mode "z": phases, "su2": arbitrary unitaries), in the basis of the rows of
    W (n, D) complex128 or at comp_rows.  Returns (F, params, block, T')."""
    prec = 0 if U.dtype == torch.complex64 else 1
    S, D = U.shape
    dc = 2 ** int(n_qubits)
    colsd = torch.tensor(list(cols), dtype=torch.int32, device=U.device)
    rows = None if comp_rows is None else torch.tensor(list(comp_rows), dtype=torch.int64,
                                                       device=U.device)
    tg = torch.tensor(np.asarray(target, dtype=np.complex128), device=U.device).contiguous()
    block = torch.empty((2, dc, dc), dtype=torch.complex128, device=U.device)
    tau = torch.zeros(1, dtype=torch.complex128, device=U.device)
    m = {"z": 1, "su2": 2}[mode]
    npar = 2 * int(n_qubits) if m == 1 else 16 * int(n_qubits)
    par = (C.c_double * npar)()
    F = C.c_double()
    check(lib().scp_fidelity_local(_ptr(U), D, S, prec, int(n_qubits), _ptr(colsd),
                                   None if W is None else _ptr(W),
                                   None if rows is None else _ptr(rows), _ptr(tg), m,
                                   _ptr(block), _ptr(tau), C.byref(F), par,
                                   None if cotangent is None else _ptr(cotangent),
                                   _stream_ptr(stream)))
    return F.value, np.array(par[:]), block[0], block[1]


def fidelity_zcomp(U, tgt: Target, n_qubits, cotangent=None, stream=None):
    """Fidelity with single-qubit phase compensation before and after the gate
    (F, phases after, phases before); fills ``cotangent`` (the costate of
    1 - F at the optimal phases) if given."""
    prec = 0 if U.dtype == torch.complex64 else 1
    S, D = U.shape
    if tgt.dc != 2 ** int(n_qubits):
        raise ValueError(f"{tgt.dc} computational states are not 2^{n_qubits}")
    block = torch.empty((tgt.dc, tgt.dc), dtype=torch.complex128, device=U.device)
    F = C.c_double()
    ph = (C.c_double * (2 * int(n_qubits)))()
    check(lib().scp_fidelity_zcomp(_ptr(U), D, S, prec, int(n_qubits), _ptr(tgt.rows),
                                   _ptr(tgt.cols), _ptr(tgt.target), _ptr(block), _ptr(tgt.tau),
                                   C.byref(F), ph, None if cotangent is None else _ptr(cotangent),
                                   _stream_ptr(stream)))
    n = int(n_qubits)
    return F.value, np.array(ph[:n]), np.array(ph[n:])


def probe_contraction(form, ops, iters, n_wg=1024, out=None, stream=None):
    """The stepper's d = 3 contraction in form 0 (VALU), 1 (MFMA 4x4x1 with the
    operand builds and moves the register layout needs) or 2 (MFMA issue
    only); ops: (nop, 18) float32 on the device.  Returns the (n_wg * 256)
    per-lane output sums (measurement only)."""
    ops = ops.contiguous()
    if out is None:
        out = torch.empty(n_wg * 256, dtype=torch.float32, device=ops.device)
    check(lib().scp_probe_contraction(int(form), int(n_wg), int(iters), int(ops.shape[0]),
                                      _ptr(ops), _ptr(out), _stream_ptr(stream)))
    return out


def padded_indices(truncs, indices):
    """Product-state indices given in the modes' own truncations (mode 0 most
    significant) mapped to the library's index space, in which every mode has
    the largest truncation d (a mode truncated to fewer levels carries inert
    extra levels that no operator reaches).  Identity when all are equal."""
    truncs = [int(v) for v in truncs]
    d = max(truncs)
    out = []
    for idx in indices:
        r, levels = int(idx), []
        for t in reversed(truncs):
            levels.append(r % t)
            r //= t
        if r:
            raise ValueError(f"index {idx} outside the product space {truncs}")
        v = 0
        for a in reversed(levels):
            v = v * d + a
        out.append(v)
    return out


def basis_columns(D, columns, dtype=torch.complex64, device="cuda"):
    psi0 = torch.zeros((len(columns), D), dtype=dtype, device=device)
    for j, c in enumerate(columns):
        psi0[j, c] = 1.0
    return psi0
