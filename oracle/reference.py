"""Python side of the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parameters are read by
attribute from any object that carries them (mesh: ``n, lo, hi, dirichlet``;
coefficients: ``k_l, k_g, rc_l, rc_g, rho_l, rho_g, mu_l, mu_g, alpha_m,
alpha_k, alpha_c, alpha_v, heaviside, eps``); missing attributes default to 0.

Operators (paper Sec. 2.1, 2.3; App. B):
  heat:  A = alpha_m M(rc) + alpha_k K(k)        (eq. heat_transfer, backward Euler)
  Oseen: A = alpha_m M(rho) + alpha_c C(rho, u0) + alpha_v V(mu)   (eq. momentum_balance)
with homogeneous Dirichlet dofs as identity rows with their columns removed.
Solvers (App. B: CG for symmetric and GMRES for non-symmetric systems).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")


class OMesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("dirichlet", ctypes.c_int32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class OCoeffs(ctypes.Structure):
    _fields_ = [("heaviside", ctypes.c_int32), ("pad_", ctypes.c_int32), ("eps", ctypes.c_double),
                ("alpha_m", ctypes.c_double), ("alpha_k", ctypes.c_double),
                ("alpha_c", ctypes.c_double), ("alpha_v", ctypes.c_double),
                ("k_l", ctypes.c_double), ("k_g", ctypes.c_double),
                ("rc_l", ctypes.c_double), ("rc_g", ctypes.c_double),
                ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
                ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
                ("k_s", ctypes.c_double), ("rc_s", ctypes.c_double), ("rho_s", ctypes.c_double),
                ("mu_s", ctypes.c_double), ("T_sol", ctypes.c_double), ("T_liq", ctypes.c_double),
                ("darcy_C", ctypes.c_double), ("darcy_b", ctypes.c_double), ("penalty", ctypes.c_double)]


_lib = None


def lib():
    """Load liboracle.so, compiling it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from .build import build
            build()
        L = ctypes.CDLL(_LIBPATH)
        P, D, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64
        L.orc_csr_rowptr.restype = I64
        L.orc_prolongation.restype = I64
        for name in ["orc_gauss3", "orc_basis1d", "orc_constrained_mask", "orc_heaviside",
                     "orc_heat_cell_matrix", "orc_oseen_cell_matrix", "orc_csr_cols",
                     "orc_assemble_heat", "orc_assemble_oseen", "orc_spmv", "orc_heat_rows",
                     "orc_oseen_rows", "orc_quad_points", "orc_heat_qp_coeffs", "orc_heat_grad",
                     "orc_load_vector", "orc_heat_sources", "orc_nodal_gradient", "orc_point_values",
                     "orc_transport_velocity"]:
            getattr(L, name).restype = None
        L.orc_basis1d.argtypes = [D, P, P]
        L.orc_heaviside.argtypes = [ctypes.c_int32, D, P, P, P, I64]
        L.orc_spmv.argtypes = [I64, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def omesh(mesh) -> OMesh:
    m = OMesh()
    for d in range(3):
        m.n[d] = int(mesh.n[d])
        m.lo[d] = float(getattr(mesh, "lo", (0, 0, 0))[d])
        m.hi[d] = float(getattr(mesh, "hi", (1, 1, 1))[d])
    m.dirichlet = int(getattr(mesh, "dirichlet", 0))
    return m


def ocoeffs(params, **override) -> OCoeffs:
    c = OCoeffs()
    for name, _ in OCoeffs._fields_:
        if name == "pad_":
            continue
        v = override.get(name, getattr(params, name, 0) if params is not None else 0)
        setattr(c, name, int(v) if name == "heaviside" else float(v))
    return c


def n_nodes(mesh) -> int:
    return int(np.prod([2 * c + 1 for c in mesh.n]))


def n_cells(mesh) -> int:
    return int(np.prod(mesh.n))


# ---------------------------------------------------------------------------
# Reference element and pointwise functions
# ---------------------------------------------------------------------------

def gauss3():
    xi = np.zeros(3)
    w = np.zeros(3)
    lib().orc_gauss3(_p(xi), _p(w))
    return xi, w


def basis1d(xi: float):
    v = np.zeros(3)
    d = np.zeros(3)
    lib().orc_basis1d(float(xi), _p(v), _p(d))
    return v, d


def heaviside(phi, kind: int = 0, eps: float = 0.0):
    """Smoothed Heaviside H(phi) and dH/dphi (Sec. 2.3, eq. heaviside; kind 0 is
    the linear form H = (1+phi)/2 clamped to [0,1])."""
    phi = _f64(np.atleast_1d(phi))
    H = np.zeros_like(phi)
    dH = np.zeros_like(phi)
    lib().orc_heaviside(int(kind), float(eps), _p(phi), _p(H), _p(dH), phi.size)
    return H, dH


def constrained_mask(mesh) -> np.ndarray:
    m = omesh(mesh)
    mask = np.zeros(n_nodes(mesh), dtype=np.uint8)
    lib().orc_constrained_mask(ctypes.byref(m), _p(mask))
    return mask.astype(bool)


def heat_cell_matrix(X8x3, params, phi27=None, kq27=None, rcq27=None, u0_3x27=None, Tc27=None,
                     **override) -> np.ndarray:
    """Heat cell matrix; u0_3x27 (nodal velocity of the cell) adds the convective
    term, Tc27 (nodal temperature of the cell) selects the three-phase coefficients."""
    X = _f64(X8x3).reshape(8, 3)
    Ae = np.zeros((27, 27))
    c = ocoeffs(params, **override)
    lib().orc_heat_cell_matrix(_p(X), ctypes.byref(c), _p(None if phi27 is None else _f64(phi27)),
                               _p(None if kq27 is None else _f64(kq27)),
                               _p(None if rcq27 is None else _f64(rcq27)),
                               _p(None if u0_3x27 is None else _f64(u0_3x27)),
                               _p(None if Tc27 is None else _f64(Tc27)), _p(Ae))
    return Ae


def oseen_cell_matrix(X8x3, params, phi27, u0_3x27, Tc27=None, **override) -> np.ndarray:
    X = _f64(X8x3).reshape(8, 3)
    Ae = np.zeros((81, 81))
    c = ocoeffs(params, **override)
    lib().orc_oseen_cell_matrix(_p(X), ctypes.byref(c), _p(_f64(phi27)), _p(_f64(u0_3x27)),
                                _p(None if Tc27 is None else _f64(Tc27)), _p(Ae))
    return Ae


def unit_cell_vertices(h=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    X = np.zeros((8, 3))
    for v in range(8):
        for d in range(3):
            X[v, d] = origin[d] + h[d] * ((v >> d) & 1)
    return X


# ---------------------------------------------------------------------------
# Assembly
# ---------------------------------------------------------------------------

def _pattern(mesh, ncomp: int):
    m = omesh(mesh)
    nrows = ncomp * n_nodes(mesh)
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    nnz = lib().orc_csr_rowptr(ctypes.byref(m), ncomp, _p(rowptr))
    cols = np.zeros(nnz, dtype=np.int32)
    lib().orc_csr_cols(ctypes.byref(m), ncomp, _p(rowptr), _p(cols))
    return m, rowptr, cols


def heat_matrix(mesh, params, phi=None, kq=None, rcq=None, u0=None, Tc=None, **override) -> sp.csr_matrix:
    """Global heat matrix (CSR), coefficients from nodal phi or from per-qp arrays;
    a nodal velocity u0 ([3][n_nodes]) adds the convective term, a nodal
    temperature Tc selects the three-phase coefficients."""
    m, rowptr, cols = _pattern(mesh, 1)
    vals = np.zeros(cols.size)
    c = ocoeffs(params, **override)
    phi = None if phi is None else _f64(phi)
    kq = None if kq is None else _f64(kq)
    rcq = None if rcq is None else _f64(rcq)
    u0 = None if u0 is None else _f64(u0)
    Tc = None if Tc is None else _f64(Tc)
    lib().orc_assemble_heat(ctypes.byref(m), ctypes.byref(c), _p(phi), _p(kq), _p(rcq), _p(u0), _p(Tc),
                            _p(rowptr), _p(cols), _p(vals))
    n = n_nodes(mesh)
    return sp.csr_matrix((vals, cols, rowptr), shape=(n, n))


def oseen_matrix(mesh, params, phi, u0, Tc=None, **override) -> sp.csr_matrix:
    m, rowptr, cols = _pattern(mesh, 3)
    vals = np.zeros(cols.size)
    c = ocoeffs(params, **override)
    lib().orc_assemble_oseen(ctypes.byref(m), ctypes.byref(c), _p(_f64(phi)), _p(_f64(u0)),
                             _p(None if Tc is None else _f64(Tc)), _p(rowptr), _p(cols), _p(vals))
    n = 3 * n_nodes(mesh)
    return sp.csr_matrix((vals, cols, rowptr), shape=(n, n))


def spmv(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = A x by the plain CSR row loop (OpenMP over rows)."""
    x = _f64(x)
    y = np.empty(A.shape[0])
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = _f64(A.data)
    lib().orc_spmv(A.shape[0], _p(indptr), _p(indices), _p(data), _p(x), _p(y))
    return y


def heat_rows(mesh, params, x, rows, phi=None, kq=None, rcq=None, u0=None, transpose=False, Tc=None,
              **override) -> np.ndarray:
    """Selected entries of y = A x (or A^T x) for the heat operator, from cell matrices only."""
    m = omesh(mesh)
    c = ocoeffs(params, **override)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    lib().orc_heat_rows(ctypes.byref(m), ctypes.byref(c), _p(None if phi is None else _f64(phi)),
                        _p(None if kq is None else _f64(kq)), _p(None if rcq is None else _f64(rcq)),
                        _p(None if u0 is None else _f64(u0)), _p(None if Tc is None else _f64(Tc)), _p(_f64(x)),
                        ctypes.c_int32(1 if transpose else 0),
                        ctypes.c_int64(rows.size), _p(rows), _p(out))
    return out


def oseen_rows(mesh, params, phi, u0, x, rows, transpose=False, Tc=None, **override) -> np.ndarray:
    m = omesh(mesh)
    c = ocoeffs(params, **override)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    lib().orc_oseen_rows(ctypes.byref(m), ctypes.byref(c), _p(_f64(phi)), _p(_f64(u0)),
                         _p(None if Tc is None else _f64(Tc)), _p(_f64(x)),
                         ctypes.c_int32(1 if transpose else 0), ctypes.c_int64(rows.size), _p(rows), _p(out))
    return out


def quad_points(mesh) -> np.ndarray:
    m = omesh(mesh)
    xq = np.zeros((n_cells(mesh) * 27, 3))
    lib().orc_quad_points(ctypes.byref(m), _p(xq))
    return xq


def load_vector(mesh, fq) -> np.ndarray:
    """b_i = int f N_i by the 3x3x3 Gauss rule, from f at the quadrature points."""
    m = omesh(mesh)
    b = np.zeros(n_nodes(mesh))
    lib().orc_load_vector(ctypes.byref(m), _p(_f64(fq)), _p(b))
    return b


def heat_qp_coeffs(mesh, params, phi, **override):
    m = omesh(mesh)
    c = ocoeffs(params, **override)
    kq = np.zeros(n_cells(mesh) * 27)
    rcq = np.zeros_like(kq)
    lib().orc_heat_qp_coeffs(ctypes.byref(m), ctypes.byref(c), _p(_f64(phi)), _p(kq), _p(rcq))
    return kq, rcq


def heat_grad(mesh, params, T, Told, lam, phi=None, dT=None, **override):
    """dL/dk_q, dL/drc_q and (with phi) dL/dphi_j for one implicit heat step,
    given the adjoint state lam.  dT = T - T_old may be passed directly."""
    m = omesh(mesh)
    c = ocoeffs(params, **override)
    dk = np.zeros(n_cells(mesh) * 27)
    drc = np.zeros_like(dk)
    dphi = np.zeros(n_nodes(mesh)) if phi is not None else None
    lib().orc_heat_grad(ctypes.byref(m), ctypes.byref(c), _p(None if phi is None else _f64(phi)),
                        _p(_f64(T)), _p(_f64(Told)), _p(None if dT is None else _f64(dT)), _p(_f64(lam)),
                        _p(dk), _p(drc), _p(dphi))
    return dk, drc, dphi


def prolongation(mesh_coarse) -> sp.csr_matrix:
    """P[i, j] = N_j^coarse(x_i^fine) from the coarse Q2 space on mesh_coarse to
    the Q2 space on the uniformly refined mesh."""
    m = omesh(mesh_coarse)
    nf = [2 * c for c in mesh_coarse.n]
    nrow = int(np.prod([2 * c + 1 for c in nf]))
    rowptr = np.zeros(nrow + 1, dtype=np.int64)
    nnz = lib().orc_prolongation(ctypes.byref(m), _p(rowptr), None, None)
    cols = np.zeros(nnz, dtype=np.int32)
    vals = np.zeros(nnz)
    lib().orc_prolongation(ctypes.byref(m), _p(rowptr), _p(cols), _p(vals))
    return sp.csr_matrix((vals, cols, rowptr), shape=(nrow, n_nodes(mesh_coarse)))


# ---------------------------------------------------------------------------
# Krylov solvers (App. B; Saad, Iterative Methods for Sparse Linear Systems)
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    rel_res: float      # true ||b - A x|| / ||b|| at exit
    converged: bool
    history: List[float]


def jacobi_cg(A, b, rtol=1e-10, maxit=10000, dinv=None, matvec=None) -> SolveResult:
    """Preconditioned CG with the diagonal (Jacobi) preconditioner, x0 = 0.

    Stops when the recursively updated residual satisfies ||r|| <= rtol ||b||;
    ``iters`` counts the products with A.  The returned ``rel_res`` is the true
    residual recomputed at exit."""
    mv = matvec or (lambda v: spmv(A, v))
    b = _f64(b)
    if dinv is None:
        dinv = 1.0 / A.diagonal()
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bn == 0.0:
        return SolveResult(x, 0, 0.0, True, [0.0])
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    hist = [1.0]
    it = 0
    conv = False
    while it < maxit:
        q = mv(p)
        it += 1
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / bn
        hist.append(rel)
        if rel <= rtol:
            conv = True
            break
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true = np.linalg.norm(b - mv(x)) / bn
    return SolveResult(x, it, true, conv, hist)


def block_jacobi(A: sp.csr_matrix, nn: int) -> Callable[[np.ndarray], np.ndarray]:
    """Point-block Jacobi for a 3-component operator (component-major dofs):
    the 3x3 block of each node, inverted."""
    B = np.zeros((nn, 3, 3))
    idx = np.arange(nn)
    for c in range(3):
        for cp in range(3):
            B[:, c, cp] = np.asarray(A[c * nn + idx, cp * nn + idx]).ravel()
    Binv = np.linalg.inv(B)

    def apply(v):
        V = v.reshape(3, nn).T  # (nn, 3)
        return np.einsum("nij,nj->ni", Binv, V).T.reshape(-1)

    apply.blocks = B
    apply.inverse = Binv
    return apply


def gmres(A, b, precond: Optional[Callable] = None, restart=30, rtol=1e-8, maxit=10000,
          matvec=None) -> SolveResult:
    """Right-preconditioned restarted GMRES(m) (Saad Alg. 9.5) with modified
    Gram-Schmidt Arnoldi and Givens rotations, x0 = 0.  Stops when the residual
    estimate |g_{j+1}| <= rtol ||b||; ``iters`` counts Arnoldi steps."""
    mv = matvec or (lambda v: spmv(A, v))
    M = precond or (lambda v: v.copy())
    b = _f64(b)
    n = b.size
    bn = np.linalg.norm(b)
    x = np.zeros(n)
    if bn == 0.0:
        return SolveResult(x, 0, 0.0, True, [0.0])
    total = 0
    hist = []
    conv = False
    while total < maxit:
        r = b - mv(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bn)
        if beta / bn <= rtol:
            conv = True
            break
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        inner_conv = False
        for j in range(m):
            w = mv(M(V[j]))
            total += 1
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w -= H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) / bn <= rtol or total >= maxit:
                inner_conv = abs(g[j + 1]) / bn <= rtol
                break
        y = scipy.linalg.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x += M(V[:j_done].T @ y)
        if inner_conv:
            true = np.linalg.norm(b - mv(x)) / bn
            if true <= rtol:
                conv = True
                break
    true = np.linalg.norm(b - mv(x)) / bn
    return SolveResult(x, total, true, conv and true <= rtol, hist)


def direct_solve(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """Exact discrete solution by sparse LU (library factorization)."""
    return spla.splu(A.tocsc()).solve(_f64(b))


# ---------------------------------------------------------------------------
# Multigrid pieces (FP64 reference of the V-cycle preconditioner)
# ---------------------------------------------------------------------------

def knuth_start_vector(n: int) -> np.ndarray:
    """Deterministic start vector for eigenvalue estimation: Knuth's
    multiplicative hash v_i = ((i * 2654435761) mod 2^32) / 2^32 - 1/2."""
    i = np.arange(n, dtype=np.uint64)
    h = (i * np.uint64(2654435761)) % np.uint64(2 ** 32)
    return h.astype(np.float64) / 2.0 ** 32 - 0.5


def lanczos_max_eig(matvec, dinv, v0, steps=12) -> float:
    """Largest eigenvalue of D^{-1} A estimated by ``steps`` Lanczos steps on the
    symmetric form D^{-1/2} A D^{-1/2} from start vector v0 (Saad Alg. 6.15):
    largest eigenvalue of the resulting tridiagonal matrix."""
    s = np.sqrt(dinv)
    q = v0 / np.linalg.norm(v0)
    q_prev = np.zeros_like(q)
    beta = 0.0
    al, be = [], []
    for k in range(steps):
        w = s * matvec(s * q)
        a = w @ q
        w = w - a * q - beta * q_prev
        al.append(a)
        beta = np.linalg.norm(w)
        if k == steps - 1 or beta == 0.0:
            break
        be.append(beta)
        q_prev, q = q, w / beta
    T = np.diag(al) + np.diag(be[:len(al) - 1], 1) + np.diag(be[:len(al) - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def chebyshev_smooth(matvec, dinv, b, x0, degree, lmin, lmax):
    """Chebyshev iteration of the given degree for A x = b preconditioned by
    D^{-1}, targeting the eigenvalue interval [lmin, lmax] of D^{-1}A
    (Saad Alg. 12.1 with the residual updated recursively).  With x0 = None the
    initial guess is zero and no product with A is needed for r0."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - matvec(x0)
    rho = 1.0 / sigma
    d = dinv * r / theta
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = r - matvec(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x


@dataclass(frozen=True)
class MeshDesc:
    """Uniform box mesh description (cells per direction, box, Dirichlet faces)."""
    n: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    dirichlet: int = 0


@dataclass
class MGLevel:
    mesh: object
    A: sp.csr_matrix
    dinv: np.ndarray
    lmax: float
    lmin: float
    P: Optional[sp.csr_matrix] = None   # from the next coarser level to this one (Dirichlet-masked)


def inject(phi_fine: np.ndarray, mesh_coarse) -> np.ndarray:
    """Coarse nodal values of a fine nodal field at the coinciding nodes
    (coarse node (I,J,K) = fine node (2I,2J,2K))."""
    nxc, nyc, nzc = [2 * c + 1 for c in mesh_coarse.n]
    nxf, nyf, nzf = [2 * (2 * c) + 1 for c in mesh_coarse.n]
    F = phi_fine.reshape(nzf, nyf, nxf)
    return np.ascontiguousarray(F[::2, ::2, ::2]).reshape(-1)


def heat_mg_levels(mesh_fine, params, phi_fine, n_coarse=4, degree=4, smoothing_range=20.0,
                   eig_steps=12, eig_safety=1.2, lmax_override: Optional[Sequence[float]] = None):
    """Level hierarchy of the heat operator from the fine mesh down to n_coarse
    cells per direction.  Each level is rediscretized with the injected level
    set; P is the Q2 embedding with rows and columns of constrained nodes
    zeroed; Chebyshev bounds lmax = eig_safety * Lanczos estimate,
    lmin = lmax / smoothing_range.  Index 0 is the coarsest level."""
    meshes = []
    m = mesh_fine
    phis = []
    phi = _f64(phi_fine)
    while True:
        meshes.append(m)
        phis.append(phi)
        if m.n[0] <= n_coarse:
            break
        mc = MeshDesc(tuple(c // 2 for c in m.n), tuple(m.lo), tuple(m.hi), int(m.dirichlet))
        phi = inject(phi, mc)
        m = mc
    meshes = meshes[::-1]
    phis = phis[::-1]
    levels = []
    for li, (m, ph) in enumerate(zip(meshes, phis)):
        A = heat_matrix(m, params, phi=ph)
        dinv = 1.0 / A.diagonal()
        if lmax_override is not None:
            lmax = float(lmax_override[li])
        else:
            lmax = eig_safety * lanczos_max_eig(lambda v: spmv(A, v), dinv, knuth_start_vector(A.shape[0]),
                                                eig_steps)
        P = None
        if li > 0:
            Pm = prolongation(meshes[li - 1])
            cf = constrained_mask(m)
            cc = constrained_mask(meshes[li - 1])
            Pm = sp.diags((~cf).astype(float)) @ Pm @ sp.diags((~cc).astype(float))
            P = Pm.tocsr()
        levels.append(MGLevel(m, A, dinv, lmax, lmax / smoothing_range, P))
    return levels


def vcycle(levels: List[MGLevel], b: np.ndarray, degree=4, coarse_solve=None, level=None) -> np.ndarray:
    """One V-cycle z = V(b): Chebyshev pre-smoothing from zero, residual,
    restriction R = P^T, recursive coarse correction, prolongation, Chebyshev
    post-smoothing; the coarsest level is solved exactly."""
    if level is None:
        level = len(levels) - 1
    L = levels[level]
    if level == 0:
        if coarse_solve is not None:
            return coarse_solve(b)
        return direct_solve(L.A, b)
    mv = lambda v: spmv(L.A, v)
    x = chebyshev_smooth(mv, L.dinv, b, None, degree, L.lmin, L.lmax)
    r = b - mv(x)
    rc = L.P.T @ r
    ec = vcycle(levels, rc, degree, coarse_solve, level - 1)
    x = x + L.P @ ec
    x = chebyshev_smooth(mv, L.dinv, b, x, degree, L.lmin, L.lmax)
    return x


def flexible_cg(A, b, precond, rtol=1e-8, maxit=1000, matvec=None) -> SolveResult:
    """Flexible preconditioned CG (Notay 2000) with the Polak-Ribiere choice
    beta = r_{k+1}.(z_{k+1} - z_k) / r_k.z_k, x0 = 0."""
    mv = matvec or (lambda v: spmv(A, v))
    b = _f64(b)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = r @ z
    hist = [1.0]
    it = 0
    conv = False
    while it < maxit:
        q = mv(p)
        it += 1
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / bn
        hist.append(rel)
        if rel <= rtol:
            conv = True
            break
        z_new = precond(r)
        rz_new = r @ z_new
        beta = (rz_new - r @ z) / rz
        z = z_new
        rz = rz_new
        p = z + beta * p
    true = np.linalg.norm(b - mv(x)) / bn
    return SolveResult(x, it, true, conv, hist)


# ---------------------------------------------------------------------------
# Interface heat sources
# ---------------------------------------------------------------------------

class OSources(ctypes.Structure):
    _fields_ = [("terms", ctypes.c_int32), ("pad_", ctypes.c_int32), ("evap_coeff", ctypes.c_double),
                ("molar_mass", ctypes.c_double), ("vapor_density", ctypes.c_double), ("T_boil", ctypes.c_double),
                ("h_v", ctypes.c_double), ("power", ctypes.c_double), ("absorptivity", ctypes.c_double),
                ("radius", ctypes.c_double), ("focus", ctypes.c_double * 3), ("dir", ctypes.c_double * 3)]


def osources(sp) -> OSources:
    o = OSources()
    o.terms = int(sp.terms)
    for name in ["evap_coeff", "molar_mass", "vapor_density", "T_boil", "h_v", "power", "absorptivity", "radius"]:
        setattr(o, name, float(getattr(sp, name)))
    for d in range(3):
        o.focus[d] = float(sp.focus[d])
        o.dir[d] = float(sp.dir[d])
    return o


def heat_sources(mesh, params, sources, phi, T, **override) -> np.ndarray:
    """Heat right-hand side of the interface fluxes (evaporative cooling and the
    laser heat flux) from nodal phi and T; zero on Dirichlet nodes."""
    m = omesh(mesh)
    c = ocoeffs(params, **override)
    s = osources(sources)
    b = np.zeros(n_nodes(mesh))
    lib().orc_heat_sources(ctypes.byref(m), ctypes.byref(c), ctypes.byref(s), _p(_f64(phi)), _p(_f64(T)), _p(b))
    return b


# ---------------------------------------------------------------------------
# Whole implicit heat steps with the Dirichlet nodes held at T_old
# ---------------------------------------------------------------------------

def without_dirichlet(mesh) -> MeshDesc:
    """The same mesh with no Dirichlet faces: every column of the operator present."""
    return MeshDesc(tuple(int(c) for c in mesh.n), tuple(getattr(mesh, "lo", (0.0, 0.0, 0.0))),
                    tuple(getattr(mesh, "hi", (1.0, 1.0, 1.0))), 0)


def heat_step(mesh, params, T_old, phi=None, kq=None, rcq=None, delta=True):
    """One backward-Euler step of the heat equation (Sec. 2.1, eq. heat_transfer)
    with the Dirichlet nodes held at T_old; on the free rows

        alpha_m M (T - T_old) + alpha_k K T = 0,    T = T_old on Dirichlet nodes,

    with M and K assembled on the mesh without Dirichlet faces (every column
    present) and the free block solved by sparse LU.

    delta=False solves for T itself:  A_ff T_f = (alpha_m M T_old)_f - A_fD T_old_D.
    delta=True solves for dT = T - T_old:  A_ff dT_f = -(alpha_k K T_old)_f, which
    avoids the cancellation of forming T - T_old at small time steps.
    Returns (T, dT)."""
    T_old = _f64(T_old)
    m0 = without_dirichlet(mesh)
    free = ~constrained_mask(mesh)
    A = heat_matrix(m0, params, phi=phi, kq=kq, rcq=rcq).tocsr()
    Aff = A[free][:, free]
    if delta:
        K = heat_matrix(m0, params, phi=phi, kq=kq, rcq=rcq, alpha_m=0.0)
        dT = np.zeros_like(T_old)
        dT[free] = direct_solve(Aff, -(K @ T_old)[free])
        return T_old + dT, dT
    M = heat_matrix(m0, params, phi=phi, kq=kq, rcq=rcq, alpha_k=0.0)
    T = T_old.copy()
    rhs = (M @ T_old)[free] - A[free][:, ~free] @ T_old[~free]
    T[free] = direct_solve(Aff, rhs)
    return T, T - T_old


@dataclass
class PicardResult:
    T: np.ndarray
    iterations: int
    converged: bool
    updates: List[float]


def picard_step(mesh, params, phi, T_old, sources=None, tol=1e-11, maxit=40) -> PicardResult:
    """One implicit heat step with temperature-dependent three-phase coefficients
    (Sec. 4.1-4.3), the Tanasawa penalty R of params.penalty (App. C) and the
    interface sources b (Sec. 2.4, Sec. 4; None: none):

        alpha_m M(T) (T - T_old) + K(T) T + R T = b(T)  on the free rows,
        T = T_old on Dirichlet nodes,

    by Picard iteration: with the coefficients and b frozen at T^k, solve the
    linear step for dT = T^{k+1} - T_old on the free rows,
        (alpha_m M + K + R)(T^k)_ff dT_f = (b(T^k) - (K + R)(T^k) T_old)_f,
    with every column present (assembled on the mesh without Dirichlet faces),
    by sparse LU, until ||T^{k+1} - T^k|| <= tol ||T^{k+1}||."""
    T_old = _f64(T_old)
    m0 = without_dirichlet(mesh)
    free = ~constrained_mask(mesh)
    T = T_old.copy()
    updates = []
    for k in range(maxit):
        A = heat_matrix(m0, params, phi=phi, Tc=T).tocsr()
        KR = heat_matrix(m0, params, phi=phi, Tc=T, alpha_m=0.0)
        b = heat_sources(mesh, params, sources, phi, T) if sources is not None else np.zeros_like(T)
        Tn = T_old.copy()
        Tn[free] += direct_solve(A[free][:, free], (b - KR @ T_old)[free])
        upd = float(np.linalg.norm(Tn - T) / np.linalg.norm(Tn))
        updates.append(upd)
        T = Tn
        if upd <= tol:
            return PicardResult(T, k + 1, True, updates)
    return PicardResult(T, maxit, False, updates)


# ---------------------------------------------------------------------------
# Level-set transport velocity (Sec. 2.5, App. A)
# ---------------------------------------------------------------------------

def nodal_gradient(mesh, f) -> np.ndarray:
    """Gradient of the Q2 interpolant of nodal f at every node, averaged over
    the cells containing the node; shape (3, n_nodes)."""
    m = omesh(mesh)
    g = np.zeros(3 * n_nodes(mesh))
    lib().orc_nodal_gradient(ctypes.byref(m), _p(_f64(f)), _p(g))
    return g.reshape(3, -1)


def point_values(mesh, f, x) -> np.ndarray:
    """Values of the Q2 interpolant of nodal f at points x (shape (np, 3)),
    each moved to the nearest point of the box first."""
    m = omesh(mesh)
    x = _f64(np.asarray(x).reshape(-1, 3))
    out = np.zeros(x.shape[0])
    lib().orc_point_values(ctypes.byref(m), _p(_f64(f)), ctypes.c_int64(x.shape[0]), _p(x), _p(out))
    return out


@dataclass
class TransportVelocity:
    u_gamma: np.ndarray         # (3, n_nodes)
    normal: np.ndarray          # (3, n_nodes), into the liquid
    x_gamma: Optional[np.ndarray] = None   # (3, n_nodes), variant 2
    x_liquid: Optional[np.ndarray] = None  # (3, n_nodes), variant 2


def transport_velocity(mesh, params, sources, variant, phi, u, T, **override) -> TransportVelocity:
    """Level-set transport velocity at every node: variant 1 (eq.
    transport_vel_local_continuous) or 2 (eq. transport_vel_extension_liquid),
    the Tanasawa mass flux of ``sources`` (eq. mDotTanasawa); params carries
    heaviside, eps, rho_l, rho_g.  u: nodal velocity [3][n_nodes]."""
    m = omesh(mesh)
    c = ocoeffs(params, **override)
    s = osources(sources)
    nn = n_nodes(mesh)
    ug, nrm = np.zeros(3 * nn), np.zeros(3 * nn)
    xg = np.zeros(3 * nn) if variant == 2 else None
    xl = np.zeros(3 * nn) if variant == 2 else None
    lib().orc_transport_velocity(ctypes.byref(m), ctypes.byref(c), ctypes.byref(s), ctypes.c_int32(variant),
                                 _p(_f64(phi)), _p(_f64(u)), _p(_f64(T)), _p(ug), _p(nrm), _p(xg), _p(xl))
    sh = lambda a: None if a is None else a.reshape(3, nn)
    return TransportVelocity(sh(ug), sh(nrm), sh(xg), sh(xl))
