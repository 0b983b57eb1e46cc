"""One implicit heat step with temperature-dependent (three-phase)
coefficients, solved by Picard iteration in the library
(``mf_heat_picard_step``).

The step is backward Euler for eq. heat_transfer with the coefficients of
Sec. 4.1-4.3 (solid fraction from T, three-phase blends of k and rho c_p) and
optionally the Tanasawa penalty of App. C and interface sources (Sec. 2.4,
Sec. 4):

    alpha_m M(rc(T)) (T - T_old) + K(k(T)) T + R T = b(T)   on the free rows,

with R the penalty term beta delta_rcp T, b the source right-hand side and
the Dirichlet nodes held at T_old.  Picard: freeze the coefficients at T^k,
solve A(T^k) dT = b(T^k) - (K(T^k) + R) T_old by Jacobi-CG, set
T^{k+1} = T_old + dT, until ||T^{k+1} - T^k|| <= tol ||T^{k+1}||.  This
module only allocates the output and marshals the call.
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
    op = mf.heat_operator(ctx, params, phi=phi)
    T = torch.empty_like(T_old)
    info, updates, cg_its = mf.heat_picard_step(op, sources, T_old.contiguous(), T, tol, maxit, cg_rtol, cg_maxit)
    return PicardResult(T=T, iterations=info.iterations, converged=bool(info.converged), updates=updates,
                        cg_iterations=cg_its)
