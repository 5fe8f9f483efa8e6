"""torch.autograd front ends: U = propagate(theta) whose backward is the
library's hand-written discrete adjoint (Sec. 2.5; checkpoints every
ceil(sqrt(N)) steps), and U = propagate_trotter(theta) (the product formulas,
complex FP64) whose backward is the local continuous adjoint of Sec. 2.5,
started from the forward's final state: nothing but U is kept between the
two passes.

theta holds the gradient parameters in the library's order: drive
parameters (drive order, then parameter order), then (E_J, E_C, E_L) of every
mode, then g of every coupling.  They enter through the system description,
which is rebuilt for the theta of each forward call.  The frame energies and
the carriers are frozen at the nominal build: they define the interaction
picture and are inputs of the method, not parameters.

PyTorch hands the backward 2 dL/dU* for a real loss of complex U; the library
takes dL/dU*, so the cotangent is halved.  The backward returns dL/dtheta
(FP64 from the library, cast to theta's dtype and device); psi0 gets no
gradient.  The RK4 adjoint exists for the FP32 path (complex64 psi0), the
product-formula adjoint for complex128 psi0.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from .api import System


class Model:
    """A description with its frame energies and carriers frozen at the
    nominal parameters, and the map theta -> description."""

    def __init__(self, desc):
        base = System(desc)
        try:
            self.desc = copy.deepcopy(desc)
            for m, md in enumerate(self.desc["modes"]):
                md["frame_eps"] = [float(v) for v in base.mode(m)["frame"]]
            om = base.carriers()
            for k, dr in enumerate(self.desc["drives"]):
                dr["omega_d"] = float(om[k])
            self.n_params = base.n_params
            self.D = base.D
        finally:
            base.close()
        self.theta0 = self.params_of(self.desc)

    @staticmethod
    def params_of(desc):
        th = []
        for dr in desc["drives"]:
            th += [float(v) for v in dr["params"]]
        for md in desc["modes"]:
            th += [float(md.get("EJ", 0.0)), float(md.get("EC", 0.0)), float(md.get("EL", 0.0))]
        for c in desc["couplings"]:
            th.append(float(c["g"]))
        return np.array(th, dtype=np.float64)

    def desc_at(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        if theta.shape != (self.n_params,):
            raise ValueError(f"theta has shape {theta.shape}, expected ({self.n_params},)")
        d = copy.deepcopy(self.desc)
        i = 0
        for dr in d["drives"]:
            n = len(dr["params"])
            dr["params"] = [float(v) for v in theta[i:i + n]]
            i += n
        for md in d["modes"]:
            md["EJ"], md["EC"], md["EL"] = (float(v) for v in theta[i:i + 3])
            i += 3
        for c in d["couplings"]:
            c["g"] = float(theta[i])
            i += 1
        return d


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, psi0, model):
        if psi0.dtype != torch.complex64:
            raise ValueError("the adjoint exists for the FP32 path: psi0 must be complex64")
        g = System(model.desc_at(theta.detach().cpu().numpy()))
        opts = g.opts(psi0.shape[0], with_ckpt=1)
        ws = g.workspace(opts, with_grad=True, device=psi0.device)
        U = g.propagate(psi0.detach().contiguous(), opts=opts, workspace=ws)
        ctx.solve = (g, opts, ws)
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return U

    @staticmethod
    def backward(ctx, gU):
        g, opts, ws = ctx.solve
        cot = (0.5 * gU).to(torch.complex64).contiguous()
        grad = g.adjoint(cot, opts, ws)
        g.close()
        ctx.solve = None
        return torch.as_tensor(grad, dtype=ctx.theta_dtype, device=ctx.theta_device), None, None


def propagate(model: Model, theta: torch.Tensor, psi0: torch.Tensor) -> torch.Tensor:
    """U (S, D) complex64 for parameters theta; differentiable in theta."""
    return _Propagate.apply(theta, psi0, model)


class _PropagateTrotter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, psi0, model, order):
        if psi0.dtype != torch.complex128:
            raise ValueError("the product formulas run in complex FP64: psi0 must be complex128")
        g = System(model.desc_at(theta.detach().cpu().numpy()))
        try:
            U = g.propagate_trotter(psi0.detach().contiguous(), order)
        except BaseException:
            g.close()
            raise
        ctx.solve = (g, order)
        # the walk back starts from exactly this state: an in-place change of
        # U before the backward is reported by autograd
        ctx.save_for_backward(U)
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return U

    @staticmethod
    def backward(ctx, gU):
        g, order = ctx.solve
        (U,) = ctx.saved_tensors
        cot = (0.5 * gU).to(torch.complex128).contiguous()
        try:
            grad = g.trotter_adjoint_final(U, cot, order)
        finally:
            g.close()
            ctx.solve = None
        return (torch.as_tensor(grad, dtype=ctx.theta_dtype, device=ctx.theta_device),
                None, None, None)


def propagate_trotter(model: Model, theta: torch.Tensor, psi0: torch.Tensor,
                      order: str = "q2") -> torch.Tensor:
    """psi_I(T) (S, D) complex128 of the product formula ``order`` ("q1",
    "q2", "q4", "q4j") for parameters theta; differentiable in theta through
    the local continuous adjoint."""
    return _PropagateTrotter.apply(theta, psi0, model, order)
