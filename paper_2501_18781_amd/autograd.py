"""Differentiable implicit heat step through the C ABI.

One backward-Euler step of the heat equation (Sec. 2.1, eq. heat_transfer
without convection), with coefficients blended through the level set
(Sec. 2.3):  A(k, rc) T = alpha_m M(rc) T_old on the free rows, with the
Dirichlet nodes held at T_old.

Forward (``mf_heat_step``) solves the delta form A dT = -alpha_k K(k) T_old
by Jacobi-CG and returns T = T_old + dT and dT (forming T - T_old afterwards
would lose about eight digits: the step changes T by ~1e-7 relative at
dt = 1e-3).  Backward (``mf_heat_step_adjoint``) solves the adjoint
A lam = dL/dT + dL/d(dT) (A is symmetric) and forms
    dL/dk_q   = -alpha_k W_q grad(lam).grad(T)
    dL/drc_q  = -alpha_m W_q lam dT
    dL/dphi_j = sum_q N_j(x_q) H'(phi_q) [(k_l - k_g) dL/dk_q + (rc_l - rc_g) dL/drc_q]
    dL/dT_old = dL/dT - alpha_k K lam
Every step runs in the library; this module only allocates the output
tensors and marshals the calls.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import mf


@dataclass
class HeatStep:
    """The fixed part of the problem: mesh context, material data, solver tolerance."""

    ctx: mf.Context
    params: object
    rtol: float = 1e-14
    maxit: int = 20000

    def operator(self, phi=None, k_q=None, rc_q=None, **override) -> mf.Operator:
        return mf.heat_operator(self.ctx, self.params, phi=phi, k_q=k_q, rc_q=rc_q, **override)

    def check(self, info: mf.SolveInfo, what: str):
        if not info.converged and info.rel_res > 1e3 * self.rtol:
            raise mf.MFError(info.status, f"heat step {what} did not converge: {info}")


class _HeatStepFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, step: HeatStep, T_old, k_q, rc_q, phi):
        op = step.operator(phi=phi, k_q=k_q, rc_q=rc_q)
        T = torch.empty_like(T_old)
        dT = torch.empty_like(T_old)
        step.check(mf.heat_step(op, T_old.contiguous(), T, dT, step.rtol, step.maxit), "solve")
        fctx.step = step
        fctx.mode_phi = phi is not None
        fctx.save_for_backward(T, dT, k_q if k_q is not None else T, rc_q if rc_q is not None else T,
                               phi if phi is not None else T)
        return T, dT

    @staticmethod
    def backward(fctx, gT, gdT):
        step = fctx.step
        T, dT, k_q, rc_q, phi = fctx.saved_tensors
        op = step.operator(phi=phi) if fctx.mode_phi else step.operator(k_q=k_q, rc_q=rc_q)
        nq = step.ctx.n_cells * 27
        want_coef = fctx.needs_input_grad[4] if fctx.mode_phi else any(fctx.needs_input_grad[2:4])
        dk = drc = dphi = None
        if want_coef and fctx.mode_phi:
            dphi = torch.empty_like(T)
        elif want_coef:
            dk = torch.empty(nq, dtype=torch.float64, device=T.device)
            drc = torch.empty_like(dk)
        gTold = torch.empty_like(T) if fctx.needs_input_grad[1] else None
        info = mf.heat_step_adjoint(op, T, dT, None if gT is None else gT.contiguous(),
                                    None if gdT is None else gdT.contiguous(), step.rtol, step.maxit,
                                    dk=dk, drc=drc, dphi=dphi, gT_old=gTold)
        step.check(info, "adjoint solve")
        return None, gTold, dk, drc, dphi


def heat_step(step: HeatStep, T_old: torch.Tensor, k_q=None, rc_q=None, phi=None):
    """(T, dT) after one implicit step; differentiable in T_old and either
    (k_q, rc_q) per quadrature point or the nodal level set phi."""
    if (phi is None) == (k_q is None):
        raise ValueError("give either phi or (k_q, rc_q)")
    return _HeatStepFn.apply(step, T_old, k_q, rc_q, phi)
