"""One implicit heat step with temperature-dependent (three-phase)
coefficients, solved by Picard iteration over the C ABI.

The step is backward Euler for eq. heat_transfer with the coefficients of
Sec. 3.2-3.3 (solid fraction from T, three-phase blends of k and rho c_p) and
optionally the Tanasawa penalty of App. C and interface sources (Sec. 2.4,
Sec. 4):

    alpha_m M(rc(T)) (T - T_old) + K(k(T)) T + R T = b(T),

with R the penalty term beta delta_rcp T and b the source right-hand side.
Picard: freeze the coefficients at T^k, solve the linear system for T^{k+1}
in delta form,

    A(T^k) dT = b(T^k) - (K(T^k) + R) T_old,   T^{k+1} = T_old + dT,

with A = alpha_m M + K + R (symmetric: Jacobi-CG), until
||T^{k+1} - T^k|| <= tol ||T^{k+1}||.  Every product, source assembly and
solve runs in the library; this module only orders the calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import mf


@dataclass
class PicardResult:
    T: torch.Tensor
    iterations: int
    converged: bool
    updates: list = field(default_factory=list)  # ||T^{k+1} - T^k|| / ||T^{k+1}||
    cg_iterations: list = field(default_factory=list)


def heat_step(ctx: mf.Context, params, phi: torch.Tensor, T_old: torch.Tensor, sources=None, tol: float = 1e-10,
              maxit: int = 30, cg_rtol: float = 1e-13, cg_maxit: int = 2000) -> PicardResult:
    """Picard iteration for one implicit three-phase heat step (module docstring).
    params: heat parameters (k_*, rc_*, T_sol, T_liq, penalty, dt, heaviside,
    eps); sources: SourceParams-like object or None (no right-hand side)."""
    T = T_old.clone()
    b = torch.zeros_like(T_old)
    kr = torch.empty_like(T_old)
    rhs = torch.empty_like(T_old)
    dT = torch.empty_like(T_old)
    res = PicardResult(T=T, iterations=0, converged=False)
    for k in range(maxit):
        op = mf.heat_operator(ctx, params, phi=phi, T_coef=T)
        if sources is not None:
            mf.heat_source_rhs(op, sources, T, b)
        mf.operator_apply(op.with_alphas(alpha_m=0.0), T_old, kr)
        torch.sub(b, kr, out=rhs)
        info = mf.cg_solve(op, rhs, dT, cg_rtol, cg_maxit)
        res.cg_iterations.append(info.iters)
        Tn = T_old + dT
        upd = float(torch.linalg.norm(Tn - T) / torch.linalg.norm(Tn))
        res.updates.append(upd)
        T = Tn
        res.iterations = k + 1
        if upd <= tol:
            res.converged = True
            break
    res.T = T
    return res
