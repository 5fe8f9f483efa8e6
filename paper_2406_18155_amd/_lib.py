"""ctypes declarations of the libscprop C ABI (include/scprop.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscprop.so")

SCP_OK, SCP_EINVAL, SCP_ENOMEM, SCP_EDEGENERATE, SCP_ENONFINITE, SCP_EHIP, SCP_EBUSY = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SCP_OK", -1: "SCP_EINVAL", -2: "SCP_ENOMEM", -3: "SCP_EDEGENERATE",
                -4: "SCP_ENONFINITE", -5: "SCP_EHIP", -6: "SCP_EBUSY"}
MODE_KIND = {"transmon": 0, "fluxonium": 1, "raw": 2}
OP = {"n": 0, "phi": 1}
ENV = {"gauss": 0, "gauss_basis": 1, "cos_ramp": 2, "const": 3, "pwc": 4}
MAX_TRUNC = 8


class ModeDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("basis_dim", C.c_int32), ("trunc", C.c_int32),
                ("has_frame", C.c_int32), ("EC", C.c_double), ("EJ", C.c_double),
                ("EL", C.c_double), ("ng", C.c_double), ("phiext", C.c_double),
                ("raw_eps", C.POINTER(C.c_double)), ("raw_ops", C.POINTER(C.c_double)),
                ("frame_eps", C.c_double * MAX_TRUNC)]


class CouplingDesc(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("op_i", C.c_int32), ("op_j", C.c_int32),
                ("g", C.c_double)]


class DriveDesc(C.Structure):
    _fields_ = [("mode", C.c_int32), ("op", C.c_int32), ("env", C.c_int32), ("n_par", C.c_int32),
                ("has_omega", C.c_int32), ("pad_", C.c_int32), ("omega_d", C.c_double),
                ("phase", C.c_double), ("sigma", C.c_double), ("par", C.POINTER(C.c_double))]


class SystemDesc(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("n_couplings", C.c_int32), ("n_drives", C.c_int32),
                ("n_steps", C.c_int32), ("T", C.c_double), ("modes", C.POINTER(ModeDesc)),
                ("couplings", C.POINTER(CouplingDesc)), ("drives", C.POINTER(DriveDesc))]


class SolveOpts(C.Structure):
    _fields_ = [("n_cols", C.c_int32), ("precision", C.c_int32), ("ckpt_every", C.c_int32),
                ("with_ckpt", C.c_int32), ("workspace_bytes", C.c_size_t)]


EXPORTS = {
    "scp_build_system": (C.c_int, [C.POINTER(SystemDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "scp_system_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "scp_system_mode": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "scp_system_carriers": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "scp_system_frame": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "scp_energy_tensor": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "scp_trotter_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)]),
    "scp_propagate_trotter": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "scp_trotter_adjoint_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                                     C.POINTER(C.c_size_t)]),
    "scp_propagate_trotter_adjoint": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                                C.c_size_t, C.c_void_p, C.c_void_p,
                                                C.POINTER(C.c_double), C.c_void_p]),
    "scp_propagate_trotter_adjoint_final": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                                      C.c_void_p, C.c_size_t, C.c_void_p,
                                                      C.c_void_p, C.POINTER(C.c_double),
                                                      C.c_void_p]),
    "scp_lindblad_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "scp_propagate_lindblad": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    "scp_lindblad_adjoint_workspace_size": (C.c_int, [C.c_void_p, C.c_int32,
                                                      C.POINTER(C.c_size_t)]),
    "scp_lindblad_adjoint": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_double), C.c_void_p]),
    "scp_fidelity_channel": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                       C.c_void_p]),
    "scp_static_zz": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.c_void_p]),
    "scp_fidelity_states": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_double), C.c_void_p]),
    "scp_eigenbasis_states": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double), C.c_double, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                        C.c_void_p]),
    "scp_fidelity_local": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    "scp_fidelity_zcomp": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p,
                                     C.c_void_p]),
    "scp_system_set_frame": (C.c_int, [C.c_void_p, C.c_int32]),
    "scp_system_set_engine": (C.c_int, [C.c_void_p, C.c_int32]),
    "scp_solve_engine": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32,
                                   C.POINTER(C.c_int32)]),
    "scp_system_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "scp_system_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                          C.POINTER(C.c_int32)]),
    "scp_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32,
                                     C.POINTER(C.c_size_t)]),
    "scp_apply_generator": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_int32, C.c_void_p]),
    "scp_propagate": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    "scp_fidelity": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(C.c_double), C.c_void_p]),
    "scp_propagate_adjoint": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "scp_propagate_adjoint_noalloc": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p,
                                                C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "scp_probe_contraction": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "scp_destroy": (None, [C.c_void_p]),
    "scp_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_double, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "scp_server_submit": (C.c_int, [C.c_void_p, C.POINTER(SystemDesc), C.POINTER(C.c_int64),
                                    C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                    C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                    C.POINTER(C.c_int64)]),
    "scp_request_bytes": (C.c_int, [C.POINTER(SystemDesc), C.c_int32, C.c_int32,
                                    C.POINTER(C.c_size_t)]),
    "scp_server_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "scp_server_result": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "scp_server_set_engine": (C.c_int, [C.c_void_p, C.c_int32]),
    "scp_server_destroy": (None, [C.c_void_p]),
    "scp_last_error": (C.c_char_p, []),
}

_lib = None


class ScpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Load libscprop.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libscprop.so not built at {LIB_PATH}; run "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != SCP_OK:
        msg = lib().scp_last_error()
        raise ScpError(status, msg.decode() if msg else "")
    return status
