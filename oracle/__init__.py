"""CPU FP64 oracle for the differentiable propagation path (TEST INFRASTRUCTURE).

Plain, slow, obviously-correct numpy implementation of what the HIP library
computes: single-mode Hamiltonians and their dressed truncation, the
Kronecker-structured generator, fixed-step RK4 in the interaction picture,
the gate fidelity and its discrete adjoint gradient, and (lindblad.py) the
open-system master equation with its channel fidelity and gradient.  It shares no code with
the GPU path; only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import it.  Nothing in the product path calls it.

Citations are to arXiv:2406.18155 (SuperGrad) by section / equation.
"""
from .single_mode import (build_mode, transmon_basis, fluxonium_basis,
                          displacement_matrix, dressed_truncation, mode_derivatives)
from .system import OracleSystem, build_system
from .rk4 import propagate, apply_generator
from .fidelity import fidelity, cotangent, state_fidelity, state_cotangent
from .adjoint import gradient, loss_and_grad, param_names
from .fd import fd_gradient

__all__ = [
    "build_mode", "transmon_basis", "fluxonium_basis", "displacement_matrix",
    "dressed_truncation", "mode_derivatives", "OracleSystem", "build_system",
    "propagate", "apply_generator", "fidelity", "cotangent", "state_fidelity",
    "state_cotangent", "gradient",
    "loss_and_grad", "param_names", "fd_gradient",
]
