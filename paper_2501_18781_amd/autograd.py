"""Differentiable implicit heat step through the C ABI.

One backward-Euler step of the heat equation (Sec. 2.1, eq. heat_transfer
without convection), with coefficients blended through the level set
(Sec. 2.3):  A(k, rc) T = alpha_m M(rc) T_old,  homogeneous Dirichlet
conditions on the mesh's Dirichlet faces (T_old must vanish there).

Forward solves the delta form A dT = -alpha_k K(k) T_old by Jacobi-CG and
returns T = T_old + dT (forming T - T_old afterwards would lose about eight
digits: the step changes T by ~1e-7 relative at dt = 1e-3).  Backward solves
the adjoint A^T lam = g (g restricted to the free nodes; A is symmetric) and
calls the gradient kernel:
    dL/dk_q  = -alpha_k W_q grad(lam).grad(T)
    dL/drc_q = -alpha_m W_q lam dT
    dL/dphi_j = sum_q N_j(x_q) H'(phi_q) [(k_l - k_g) dL/dk_q + (rc_l - rc_g) dL/drc_q]
    dL/dT_old = alpha_m M lam
Every step runs in the library; this module only marshals tensors.
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

    def free(self, op: mf.Operator, v: torch.Tensor) -> torch.Tensor:
        """v with its Dirichlet entries set to zero (an apply with all factors
        zero is the identity on Dirichlet rows and zero elsewhere)."""
        fixed = torch.empty_like(v)
        mf.operator_apply(op.with_alphas(alpha_m=0.0, alpha_k=0.0), v, fixed)
        return v - fixed

    def solve(self, op: mf.Operator, b: torch.Tensor) -> torch.Tensor:
        x = torch.empty_like(b)
        info = mf.cg_solve(op, b, x, self.rtol, self.maxit, precond=mf.MF_PC_JACOBI)
        if not info.converged and info.rel_res > 1e3 * self.rtol:
            raise mf.MFError(info.status, f"heat step solve did not converge: {info}")
        return x

    def delta(self, op: mf.Operator, T_old: torch.Tensor) -> torch.Tensor:
        """dT solving A dT = -alpha_k K T_old."""
        KT = torch.empty_like(T_old)
        mf.operator_apply(op.with_alphas(alpha_m=0.0), T_old, KT)
        return self.solve(op, self.free(op, -KT))


class _HeatStepFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, step: HeatStep, T_old, k_q, rc_q, phi):
        op = step.operator(phi=phi, k_q=k_q, rc_q=rc_q)
        dT = step.delta(op, T_old)
        T = T_old + dT
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
        g = torch.zeros_like(T)
        if gT is not None:
            g = g + gT
        if gdT is not None:
            g = g + gdT  # dT = T - T_old: same sensitivity to the solve
        lam = step.solve(op, step.free(op, g.contiguous()))
        nq = step.ctx.n_cells * 27
        dk = torch.empty(nq, dtype=torch.float64, device=T.device)
        drc = torch.empty_like(dk)
        dphi = torch.empty_like(T) if fctx.mode_phi else None
        mf.heat_coeff_grad(op, T, dT, lam, dk, drc, dphi)
        gTold = torch.empty_like(T)
        mf.operator_apply(op.with_alphas(alpha_k=0.0), lam, gTold)
        gTold = step.free(op, gTold)
        if gdT is not None:
            gTold = gTold - gdT
        return (None, gTold,
                None if fctx.mode_phi else dk,
                None if fctx.mode_phi else drc,
                dphi if fctx.mode_phi else None)


def heat_step(step: HeatStep, T_old: torch.Tensor, k_q=None, rc_q=None, phi=None):
    """(T, dT) after one implicit step; differentiable in T_old and either
    (k_q, rc_q) per quadrature point or the nodal level set phi."""
    if (phi is None) == (k_q is None):
        raise ValueError("give either phi or (k_q, rc_q)")
    return _HeatStepFn.apply(step, T_old, k_q, rc_q, phi)
