"""Thin Python binding of the gfx950 library ``libmf.so`` (C ABI in include/mf.h).

Argument marshalling only: descriptor structs are filled from Python objects,
torch tensors are checked (device, dtype, size, contiguity) and passed as raw
device pointers together with torch's current HIP stream.  Every step of the
computation runs in the library's kernels.  There is no fallback: if the
library is not built, or no GPU is present, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmf.so")

MF_OK, MF_NOT_CONVERGED, MF_BREAKDOWN = 0, 1, 2
MF_HEAT, MF_OSEEN = 0, 1
MF_FP64, MF_FP32 = 0, 1
MF_COEFF_LEVELSET, MF_COEFF_QUAD = 0, 1
MF_H_LINEAR, MF_H_SINE = 0, 1
MF_PC_NONE, MF_PC_JACOBI, MF_PC_BLOCK_JACOBI = 0, 1, 2

_STATUS = {0: "MF_OK", 1: "MF_NOT_CONVERGED", 2: "MF_BREAKDOWN", -1: "MF_ERR_ARG", -2: "MF_ERR_HIP",
           -3: "MF_ERR_OOM", -4: "MF_ERR_STATE"}


class MFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("dirichlet", ctypes.c_uint32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class OperatorDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("coeff_mode", ctypes.c_int32),
                ("heaviside", ctypes.c_int32), ("eps", ctypes.c_double),
                ("alpha_m", ctypes.c_double), ("alpha_k", ctypes.c_double), ("alpha_c", ctypes.c_double),
                ("alpha_v", ctypes.c_double), ("k_l", ctypes.c_double), ("k_g", ctypes.c_double),
                ("rc_l", ctypes.c_double), ("rc_g", ctypes.c_double), ("rho_l", ctypes.c_double),
                ("rho_g", ctypes.c_double), ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
                ("phi", ctypes.c_void_p), ("k_q", ctypes.c_void_p), ("rc_q", ctypes.c_void_p),
                ("u0", ctypes.c_void_p), ("k_s", ctypes.c_double), ("rc_s", ctypes.c_double),
                ("rho_s", ctypes.c_double), ("mu_s", ctypes.c_double), ("T_sol", ctypes.c_double),
                ("T_liq", ctypes.c_double), ("darcy_C", ctypes.c_double), ("darcy_b", ctypes.c_double),
                ("penalty", ctypes.c_double), ("T_coef", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("rel_res_est", ctypes.c_double)]

    def __repr__(self):
        return (f"SolveInfo(iters={self.iters}, converged={bool(self.converged)}, rel_res={self.rel_res:.3e}, "
                f"rel_res_est={self.rel_res_est:.3e})")


class MGParams(ctypes.Structure):
    _fields_ = [("coarse_cells", ctypes.c_int32), ("degree", ctypes.c_int32), ("smoothing_range", ctypes.c_double),
                ("eig_steps", ctypes.c_int32), ("eig_safety", ctypes.c_double),
                ("lambda_max", ctypes.POINTER(ctypes.c_double)), ("coarse_rtol", ctypes.c_double),
                ("coarse_maxit", ctypes.c_int32), ("auto_levels", ctypes.c_int32), ("smooth_degree", ctypes.c_int32),
                ("beta_stop", ctypes.c_double), ("lambda_min", ctypes.POINTER(ctypes.c_double))]


MF_SRC_EVAPORATION, MF_SRC_LASER, MF_SRC_PENALTY = 1, 2, 4


class SourcesDesc(ctypes.Structure):
    _fields_ = [("terms", ctypes.c_int32), ("evaporation_coefficient", ctypes.c_double),
                ("molar_mass", ctypes.c_double), ("vapor_density", ctypes.c_double),
                ("boiling_temperature", ctypes.c_double), ("latent_heat", ctypes.c_double),
                ("laser_power", ctypes.c_double), ("absorptivity", ctypes.c_double),
                ("laser_radius", ctypes.c_double), ("focus", ctypes.c_double * 3), ("direction", ctypes.c_double * 3)]


class PicardInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("cg_iterations", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("update", ctypes.c_double)]


MF_TRANSPORT_LOCAL, MF_TRANSPORT_LIQUID_EXTENSION = 1, 2


class TransportDesc(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("heaviside", ctypes.c_int32), ("eps", ctypes.c_double),
                ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
                ("evaporation_coefficient", ctypes.c_double), ("molar_mass", ctypes.c_double),
                ("vapor_density", ctypes.c_double), ("boiling_temperature", ctypes.c_double),
                ("latent_heat", ctypes.c_double)]


# Every function of the C ABI, with its argument types.
_P = ctypes.c_void_p
_SIGS = {
    "mf_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(_P)]),
    "mf_destroy": (None, [_P]),
    "mf_last_error": (ctypes.c_char_p, [_P]),
    "mf_n_nodes": (ctypes.c_int64, [_P]),
    "mf_n_cells": (ctypes.c_int64, [_P]),
    "mf_timing_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "mf_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int32]),
    "mf_operator_apply": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P, _P]),
    "mf_operator_apply_transpose": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P, _P]),
    "mf_operator_apply_noalloc": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(OperatorDesc), _P, _P, _P]),
    "mf_operator_diagonal": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P]),
    "mf_cg_solve": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), ctypes.c_int32, _P, _P, ctypes.c_double,
                                   ctypes.c_int32, ctypes.POINTER(SolveInfo), _P]),
    "mf_gmres_solve": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _P, _P, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(SolveInfo), _P]),
    "mf_mg_create": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), ctypes.POINTER(MGParams),
                                    ctypes.POINTER(_P), _P]),
    "mf_mg_destroy": (None, [_P]),
    "mf_mg_n_levels": (ctypes.c_int32, [_P]),
    "mf_mg_lambda_max": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "mf_mg_levels": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "mf_mg_vcycle": (ctypes.c_int, [_P, _P, _P, _P]),
    "mf_mg_cg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(SolveInfo), _P]),
    "mf_quad_points": (ctypes.c_int, [_P, _P, _P]),
    "mf_heat_qp_coeffs": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P, _P]),
    "mf_heat_coeff_grad": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P, _P, _P, _P, _P, _P]),
    "mf_heat_source_rhs": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), ctypes.POINTER(SourcesDesc), _P, _P,
                                          _P]),
    "mf_transport_velocity": (ctypes.c_int, [_P, ctypes.POINTER(TransportDesc), _P, _P, _P, _P, _P]),
    "mf_heat_step": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P, _P, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(SolveInfo), _P]),
    "mf_heat_step_adjoint": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), _P, _P, _P, _P, ctypes.c_double,
                                            ctypes.c_int32, _P, _P, _P, _P, ctypes.POINTER(SolveInfo), _P]),
    "mf_heat_picard_step": (ctypes.c_int, [_P, ctypes.POINTER(OperatorDesc), ctypes.POINTER(SourcesDesc), _P, _P,
                                           ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                           ctypes.POINTER(PicardInfo), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int32), _P]),
}

_lib = None


def library() -> ctypes.CDLL:
    """Load libmf.so (built in-tree by ``paper_2501_18781_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run __graft_entry__.build() or "
                               f"python -m paper_2501_18781_amd.build")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _ptr(t: Optional[torch.Tensor], n: int, dtype: torch.dtype, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t.data_ptr()


class Context:
    """One mesh on the current device (wraps mf_ctx)."""

    def __init__(self, mesh):
        L = library()
        d = mesh_desc(mesh)
        h = _P()
        st = L.mf_create(ctypes.byref(d), ctypes.byref(h))
        if st != MF_OK:
            raise MFError(st, "mf_create failed")
        self._h = h
        self.mesh = mesh
        self.n_nodes = int(L.mf_n_nodes(h))
        self.n_cells = int(L.mf_n_cells(h))

    def check(self, st: int, accept=(MF_OK,)):
        if st not in accept:
            raise MFError(st, library().mf_last_error(self._h).decode())
        return st

    def timing_enable(self, on: bool = True):
        self.check(library().mf_timing_enable(self._h, 1 if on else 0))

    def timing_read(self, reset: bool = True):
        """(summed kernel milliseconds, number of timed launches) since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.check(library().mf_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            library().mf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """An operator descriptor plus the tensors it points to (kept alive here)."""

    def __init__(self, ctx: Context, kind: int, precision: int, coeff_mode: int = MF_COEFF_LEVELSET,
                 heaviside: int = MF_H_LINEAR, eps: float = 0.0, alpha_m=0.0, alpha_k=0.0, alpha_c=0.0, alpha_v=0.0,
                 k_l=0.0, k_g=0.0, rc_l=0.0, rc_g=0.0, rho_l=1.0, rho_g=1.0, mu_l=0.0, mu_g=0.0,
                 phi=None, k_q=None, rc_q=None, u0=None, T_coef=None, k_s=0.0, rc_s=0.0, rho_s=1.0, mu_s=0.0,
                 T_sol=0.0, T_liq=1.0, darcy_C=0.0, darcy_b=1.0, penalty=0.0):
        self.ctx = ctx
        self.dtype = torch.float64 if precision == MF_FP64 else torch.float32
        nn, nq = ctx.n_nodes, ctx.n_cells * 27
        self.tensors = (phi, k_q, rc_q, u0, T_coef)
        d = OperatorDesc()
        d.kind, d.precision, d.coeff_mode, d.heaviside = kind, precision, coeff_mode, heaviside
        d.eps, d.alpha_m, d.alpha_k, d.alpha_c, d.alpha_v = eps, alpha_m, alpha_k, alpha_c, alpha_v
        d.k_l, d.k_g, d.rc_l, d.rc_g = k_l, k_g, rc_l, rc_g
        d.rho_l, d.rho_g, d.mu_l, d.mu_g = rho_l, rho_g, mu_l, mu_g
        d.phi = _ptr(phi, nn, self.dtype, "phi")
        d.k_q = _ptr(k_q, nq, self.dtype, "k_q")
        d.rc_q = _ptr(rc_q, nq, self.dtype, "rc_q")
        d.u0 = _ptr(u0, 3 * nn, self.dtype, "u0")
        d.k_s, d.rc_s, d.rho_s, d.mu_s = k_s, rc_s, rho_s, mu_s
        d.T_sol, d.T_liq, d.darcy_C, d.darcy_b, d.penalty = T_sol, T_liq, darcy_C, darcy_b, penalty
        d.T_coef = _ptr(T_coef, nn, self.dtype, "T_coef")
        self.desc = d
        self.kind = kind
        self.n_dofs = 3 * nn if kind == MF_OSEEN else nn

    def with_alphas(self, **alphas) -> "Operator":
        """Same operator with some of alpha_m, alpha_k, alpha_c, alpha_v replaced."""
        o = Operator.__new__(Operator)
        o.__dict__.update(self.__dict__)
        d = OperatorDesc()
        ctypes.pointer(d)[0] = self.desc
        for k, v in alphas.items():
            setattr(d, k, float(v))
        o.desc = d
        return o


def heat_operator(ctx: Context, params, phi=None, k_q=None, rc_q=None, precision=MF_FP64, u0=None, T_coef=None,
                  **override) -> Operator:
    """Heat operator rc/dt M + K(k) from a parameter object (k_l, k_g, rc_l,
    rc_g, alpha_m, alpha_k, heaviside, eps); with a nodal velocity u0
    ([3][n_nodes], FP64, level-set mode) it gains the convective term
    alpha_c C(rc, u0) and is no longer symmetric; with a nodal temperature
    T_coef the coefficients are the three-phase ones at that temperature
    (k_s, rc_s, T_sol, T_liq); a nonzero `penalty` adds the Tanasawa penalty."""
    g = lambda k: override.get(k, getattr(params, k))
    opt = lambda k, d: float(override.get(k, getattr(params, k, d)))
    mode = MF_COEFF_LEVELSET if phi is not None else MF_COEFF_QUAD
    ac = opt("alpha_c", 0.0) if u0 is not None else 0.0
    return Operator(ctx, MF_HEAT, precision, mode, int(g("heaviside")), float(g("eps")),
                    alpha_m=float(g("alpha_m")), alpha_k=float(g("alpha_k")), alpha_c=ac, k_l=g("k_l"),
                    k_g=g("k_g"), rc_l=g("rc_l"), rc_g=g("rc_g"), phi=phi, k_q=k_q, rc_q=rc_q, u0=u0,
                    T_coef=T_coef, k_s=opt("k_s", 0.0), rc_s=opt("rc_s", 0.0), T_sol=opt("T_sol", 0.0),
                    T_liq=opt("T_liq", 1.0), penalty=opt("penalty", 0.0))


def oseen_operator(ctx: Context, params, phi, u0, T_coef=None, **override) -> Operator:
    """Linearized momentum operator; with a nodal temperature T_coef the
    coefficients are the three-phase ones at that temperature (rho_s, mu_s,
    T_sol, T_liq) and the Darcy damping of the solid (darcy_C, darcy_b) is added."""
    g = lambda k: override.get(k, getattr(params, k))
    opt = lambda k, d: float(override.get(k, getattr(params, k, d)))
    return Operator(ctx, MF_OSEEN, MF_FP64, MF_COEFF_LEVELSET, int(g("heaviside")), float(g("eps")),
                    alpha_m=float(g("alpha_m")), alpha_c=float(g("alpha_c")), alpha_v=float(g("alpha_v")),
                    rho_l=g("rho_l"), rho_g=g("rho_g"), mu_l=g("mu_l"), mu_g=g("mu_g"), phi=phi, u0=u0,
                    T_coef=T_coef, rho_s=opt("rho_s", 1.0), mu_s=opt("mu_s", 0.0), T_sol=opt("T_sol", 0.0),
                    T_liq=opt("T_liq", 1.0), darcy_C=opt("darcy_C", 0.0), darcy_b=opt("darcy_b", 1.0))


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI without the mf_ prefix)
# ---------------------------------------------------------------------------

def operator_apply(op: Operator, x: torch.Tensor, y: torch.Tensor, stream=None):
    c = op.ctx
    c.check(library().mf_operator_apply(c._h, ctypes.byref(op.desc), _ptr(x, op.n_dofs, op.dtype, "x"),
                                        _ptr(y, op.n_dofs, op.dtype, "y"), _stream(stream)))
    return y


def mesh_desc(mesh) -> MeshDesc:
    d = MeshDesc()
    for k in range(3):
        d.n[k] = int(mesh.n[k])
        d.lo[k] = float(getattr(mesh, "lo", (0, 0, 0))[k])
        d.hi[k] = float(getattr(mesh, "hi", (1, 1, 1))[k])
    d.dirichlet = int(getattr(mesh, "dirichlet", 0))
    return d


def operator_apply_noalloc(op: Operator, x: torch.Tensor, y: torch.Tensor, stream=None):
    """y = A x through mf_operator_apply_noalloc (no context, no allocation);
    the mesh is the one of the operator's context."""
    d = mesh_desc(op.ctx.mesh)
    st = library().mf_operator_apply_noalloc(ctypes.byref(d), ctypes.byref(op.desc),
                                             _ptr(x, op.n_dofs, op.dtype, "x"), _ptr(y, op.n_dofs, op.dtype, "y"),
                                             _stream(stream))
    if st != MF_OK:
        raise MFError(st, library().mf_last_error(None).decode())
    return y


def operator_apply_transpose(op: Operator, x: torch.Tensor, y: torch.Tensor, stream=None):
    c = op.ctx
    c.check(library().mf_operator_apply_transpose(c._h, ctypes.byref(op.desc), _ptr(x, op.n_dofs, op.dtype, "x"),
                                                  _ptr(y, op.n_dofs, op.dtype, "y"), _stream(stream)))
    return y


def operator_diagonal(op: Operator, diag: torch.Tensor, stream=None):
    c = op.ctx
    n = 9 * c.n_nodes if op.kind == MF_OSEEN else c.n_nodes
    c.check(library().mf_operator_diagonal(c._h, ctypes.byref(op.desc), _ptr(diag, n, op.dtype, "diag"),
                                           _stream(stream)))
    return diag


_SOLVER_OK = (MF_OK, MF_NOT_CONVERGED, MF_BREAKDOWN)


def cg_solve(op: Operator, b: torch.Tensor, x: torch.Tensor, rtol: float, maxit: int, precond=MF_PC_JACOBI,
             stream=None) -> SolveInfo:
    c = op.ctx
    info = SolveInfo()
    st = library().mf_cg_solve(c._h, ctypes.byref(op.desc), precond, _ptr(b, op.n_dofs, torch.float64, "b"),
                               _ptr(x, op.n_dofs, torch.float64, "x"), rtol, maxit, ctypes.byref(info),
                               _stream(stream))
    c.check(st, _SOLVER_OK)
    info.status = st
    return info


def gmres_solve(op: Operator, b: torch.Tensor, x: torch.Tensor, rtol: float, maxit: int,
                precond=MF_PC_BLOCK_JACOBI, restart: int = 30, transpose: bool = False, stream=None) -> SolveInfo:
    c = op.ctx
    info = SolveInfo()
    st = library().mf_gmres_solve(c._h, ctypes.byref(op.desc), precond, restart, 1 if transpose else 0,
                                  _ptr(b, op.n_dofs, torch.float64, "b"), _ptr(x, op.n_dofs, torch.float64, "x"),
                                  rtol, maxit, ctypes.byref(info), _stream(stream))
    c.check(st, _SOLVER_OK)
    info.status = st
    return info


@dataclass
class MGConfig:
    coarse_cells: int = 4
    degree: int = 4
    smoothing_range: float = 20.0
    eig_steps: int = 12
    eig_safety: float = 1.2
    lambda_max: Optional[Sequence[float]] = None
    coarse_rtol: float = 1e-12
    coarse_maxit: int = 500
    auto_levels: bool = False
    smooth_degree: int = 2
    beta_stop: float = 1.0  # stiffness / mass ratio of the diagonal below which a level is smoothed only
    lambda_min: Optional[Sequence[float]] = None


class Multigrid:
    """FP32 geometric multigrid V-cycle for a heat operator (wraps mf_mg)."""

    def __init__(self, op: Operator, cfg: MGConfig = MGConfig(), stream=None):
        c = op.ctx
        p = MGParams()
        p.coarse_cells, p.degree, p.smoothing_range = cfg.coarse_cells, cfg.degree, cfg.smoothing_range
        p.eig_steps, p.eig_safety = cfg.eig_steps, cfg.eig_safety
        p.coarse_rtol, p.coarse_maxit = cfg.coarse_rtol, cfg.coarse_maxit
        p.auto_levels, p.smooth_degree, p.beta_stop = int(cfg.auto_levels), cfg.smooth_degree, cfg.beta_stop
        self._lmax = self._lmin = None
        if cfg.lambda_max is not None:
            self._lmax = (ctypes.c_double * len(cfg.lambda_max))(*cfg.lambda_max)
            p.lambda_max = self._lmax
        if cfg.lambda_min is not None:
            self._lmin = (ctypes.c_double * len(cfg.lambda_min))(*cfg.lambda_min)
            p.lambda_min = self._lmin
        h = _P()
        c.check(library().mf_mg_create(c._h, ctypes.byref(op.desc), ctypes.byref(p), ctypes.byref(h),
                                       _stream(stream)))
        self._h = h
        self.op = op
        self.n_levels = int(library().mf_mg_n_levels(h))

    def lambda_max(self):
        out = (ctypes.c_double * self.n_levels)()
        self.op.ctx.check(library().mf_mg_lambda_max(self._h, out))
        return list(out)

    def levels(self):
        """Per level, coarsest first: (cells per direction, Chebyshev degree (0:
        solved by CG), lambda_min, lambda_max)."""
        k = self.n_levels
        c, d = (ctypes.c_int32 * k)(), (ctypes.c_int32 * k)()
        lo, hi = (ctypes.c_double * k)(), (ctypes.c_double * k)()
        self.op.ctx.check(library().mf_mg_levels(self._h, c, d, lo, hi))
        return [(c[i], d[i], lo[i], hi[i]) for i in range(k)]

    def close(self):
        if getattr(self, "_h", None):
            library().mf_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mg_vcycle(mg: Multigrid, r: torch.Tensor, z: torch.Tensor, stream=None):
    n = mg.op.ctx.n_nodes
    mg.op.ctx.check(library().mf_mg_vcycle(mg._h, _ptr(r, n, torch.float64, "r"), _ptr(z, n, torch.float64, "z"),
                                           _stream(stream)))
    return z


def mg_cg_solve(mg: Multigrid, b: torch.Tensor, x: torch.Tensor, rtol: float, maxit: int, stream=None) -> SolveInfo:
    n = mg.op.ctx.n_nodes
    info = SolveInfo()
    st = library().mf_mg_cg_solve(mg._h, _ptr(b, n, torch.float64, "b"), _ptr(x, n, torch.float64, "x"), rtol, maxit,
                                  ctypes.byref(info), _stream(stream))
    mg.op.ctx.check(st, _SOLVER_OK)
    info.status = st
    return info


def quad_points(ctx: Context, xq: torch.Tensor, stream=None):
    ctx.check(library().mf_quad_points(ctx._h, _ptr(xq, ctx.n_cells * 27 * 3, torch.float64, "xq"), _stream(stream)))
    return xq


def heat_qp_coeffs(op: Operator, k_q: torch.Tensor, rc_q: torch.Tensor, stream=None):
    c = op.ctx
    nq = c.n_cells * 27
    c.check(library().mf_heat_qp_coeffs(c._h, ctypes.byref(op.desc), _ptr(k_q, nq, torch.float64, "k_q"),
                                        _ptr(rc_q, nq, torch.float64, "rc_q"), _stream(stream)))
    return k_q, rc_q


def heat_coeff_grad(op: Operator, T, dT, lam, dk=None, drc=None, dphi=None, stream=None):
    c = op.ctx
    nn, nq = c.n_nodes, c.n_cells * 27
    c.check(library().mf_heat_coeff_grad(c._h, ctypes.byref(op.desc), _ptr(T, nn, torch.float64, "T"),
                                         _ptr(dT, nn, torch.float64, "dT"), _ptr(lam, nn, torch.float64, "lam"),
                                         _ptr(dk, nq, torch.float64, "dk"), _ptr(drc, nq, torch.float64, "drc"),
                                         _ptr(dphi, nn, torch.float64, "dphi"), _stream(stream)))
    return dk, drc, dphi


def _sources_desc(sources) -> SourcesDesc:
    d = SourcesDesc()
    d.terms = int(sources.terms)
    d.evaporation_coefficient, d.molar_mass = float(sources.evap_coeff), float(sources.molar_mass)
    d.vapor_density, d.boiling_temperature = float(sources.vapor_density), float(sources.T_boil)
    d.latent_heat, d.laser_power = float(sources.h_v), float(sources.power)
    d.absorptivity, d.laser_radius = float(sources.absorptivity), float(sources.radius)
    for k in range(3):
        d.focus[k] = float(sources.focus[k])
        d.direction[k] = float(sources.dir[k])
    return d


def heat_source_rhs(op: Operator, sources, T: Optional[torch.Tensor], b: torch.Tensor, stream=None):
    """b = right-hand side of the interface heat fluxes (evaporative cooling,
    laser heat flux) for the level set of the heat operator op and the nodal
    temperature T.  sources: object with terms, evap_coeff, molar_mass,
    vapor_density, T_boil, h_v, power, absorptivity, radius, focus, dir."""
    c = op.ctx
    d = _sources_desc(sources)
    nn = c.n_nodes
    c.check(library().mf_heat_source_rhs(c._h, ctypes.byref(op.desc), ctypes.byref(d),
                                         _ptr(T, nn, torch.float64, "T"), _ptr(b, nn, torch.float64, "b"),
                                         _stream(stream)))
    return b


def heat_step(op: Operator, T_old: torch.Tensor, T: torch.Tensor, dT: torch.Tensor, rtol: float, maxit: int,
              stream=None) -> SolveInfo:
    """One backward-Euler heat step in delta form (mf_heat_step): writes T and dT = T - T_old."""
    c = op.ctx
    nn = c.n_nodes
    info = SolveInfo()
    st = library().mf_heat_step(c._h, ctypes.byref(op.desc), _ptr(T_old, nn, torch.float64, "T_old"),
                                _ptr(T, nn, torch.float64, "T"), _ptr(dT, nn, torch.float64, "dT"), rtol, maxit,
                                ctypes.byref(info), _stream(stream))
    c.check(st, _SOLVER_OK)
    info.status = st
    return info


def heat_step_adjoint(op: Operator, T, dT, gT, gdT, rtol: float, maxit: int, dk=None, drc=None, dphi=None,
                      gT_old=None, stream=None) -> SolveInfo:
    """Adjoint of heat_step (mf_heat_step_adjoint): gradients of a loss with
    dL/dT = gT and dL/d(dT) = gdT (None: zero) with respect to k_q, rc_q, phi
    and T_old, written into the tensors given."""
    c = op.ctx
    nn, nq = c.n_nodes, c.n_cells * 27
    f64 = torch.float64
    info = SolveInfo()
    st = library().mf_heat_step_adjoint(c._h, ctypes.byref(op.desc), _ptr(T, nn, f64, "T"), _ptr(dT, nn, f64, "dT"),
                                        _ptr(gT, nn, f64, "gT"), _ptr(gdT, nn, f64, "gdT"), rtol, maxit,
                                        _ptr(dk, nq, f64, "dk"), _ptr(drc, nq, f64, "drc"),
                                        _ptr(dphi, nn, f64, "dphi"), _ptr(gT_old, nn, f64, "gT_old"),
                                        ctypes.byref(info), _stream(stream))
    c.check(st, _SOLVER_OK)
    info.status = st
    return info


def heat_picard_step(op: Operator, sources, T_old: torch.Tensor, T: torch.Tensor, tol: float, maxit: int,
                     cg_rtol: float, cg_maxit: int, stream=None):
    """Picard iteration of one implicit three-phase heat step
    (mf_heat_picard_step); returns (PicardInfo, per-iteration updates,
    per-iteration CG iteration counts).  sources: as heat_source_rhs, or None."""
    c = op.ctx
    nn = c.n_nodes
    info = PicardInfo()
    upd = (ctypes.c_double * maxit)()
    its = (ctypes.c_int32 * maxit)()
    src = ctypes.byref(_sources_desc(sources)) if sources is not None else None
    st = library().mf_heat_picard_step(c._h, ctypes.byref(op.desc), src, _ptr(T_old, nn, torch.float64, "T_old"),
                                       _ptr(T, nn, torch.float64, "T"), tol, maxit, cg_rtol, cg_maxit,
                                       ctypes.byref(info), upd, its, _stream(stream))
    c.check(st, _SOLVER_OK)
    info.status = st
    k = info.iterations
    return info, list(upd[:k]), list(its[:k])


def transport_velocity(ctx: Context, variant: int, params, sources, phi, u, T, u_gamma, stream=None):
    """Level-set transport velocity (mf_transport_velocity): params carries
    heaviside, eps, rho_l, rho_g; sources the Tanasawa data (evap_coeff,
    molar_mass, vapor_density, T_boil, h_v)."""
    d = TransportDesc()
    d.variant, d.heaviside, d.eps = int(variant), int(params.heaviside), float(params.eps)
    d.rho_l, d.rho_g = float(params.rho_l), float(params.rho_g)
    d.evaporation_coefficient, d.molar_mass = float(sources.evap_coeff), float(sources.molar_mass)
    d.vapor_density, d.boiling_temperature = float(sources.vapor_density), float(sources.T_boil)
    d.latent_heat = float(sources.h_v)
    nn = ctx.n_nodes
    f64 = torch.float64
    ctx.check(library().mf_transport_velocity(ctx._h, ctypes.byref(d), _ptr(phi, nn, f64, "phi"),
                                              _ptr(u, 3 * nn, f64, "u"), _ptr(T, nn, f64, "T"),
                                              _ptr(u_gamma, 3 * nn, f64, "u_gamma"), _stream(stream)))
    return u_gamma
