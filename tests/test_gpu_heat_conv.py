"""GPU heat operator with the convective term (eq. heat_transfer, rc u.grad T)
vs the FP64 oracle, through the C ABI.

Bar (FP64): normwise relative error <= 1e-12 for applies, transposes and
diagonals.  At dt = 1e-3 the convective part is a fraction of a percent of
A x, so it is also checked on its own (alpha_m = alpha_k = 0).  Solves are
compared with the oracle's own GMRES (iteration counts) and with the direct
solution of the assembled system.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2501_18781_amd import mf
from paper_2501_18781_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def relerr(a, b):
    """The larger of the normwise error ||a - b|| / ||b|| and the element-wise
    error max |a - b| / max |b|: a bar on it holds for both."""
    a = a.detach().cpu().double().numpy() if isinstance(a, torch.Tensor) else a
    b = np.asarray(b, dtype=np.float64)
    d = np.asarray(a, dtype=np.float64) - b
    return float(max(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300),
                     np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)))


def conv_case(n, dirichlet, hkind=0, dt=1e-3, speed=1.0):
    mesh = W.Mesh(n, dirichlet=dirichlet)
    eps = 2.0 / max(n)
    p = W.HeatParams(heaviside=hkind, eps=eps if hkind else 0.0, dt=dt)
    return mesh, p, W.phi_sphere(mesh, 0.3, eps), speed * W.taylor_green(mesh)


# smaller than, equal to and straddling the 4x4x4 brick, with ragged tails
MESHES = [((1, 1, 1), 0), ((3, 3, 3), W.ALL_FACES), ((5, 3, 7), W.FACE_XLO | W.FACE_ZHI),
          ((9, 9, 9), W.ALL_FACES), ((8, 8, 8), 0), ((17, 10, 5), W.FACE_YHI | W.FACE_XHI)]


@pytest.mark.parametrize("n,dirichlet", MESHES)
def test_conv_apply_and_transpose_match_oracle(gpu, n, dirichlet):
    mesh, p, phi, u0 = conv_case(n, dirichlet)
    print(f"conv heat apply n={n} dirichlet={dirichlet}", flush=True)
    x = W.uniform(0, mesh.n_nodes)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0))
    y = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    A = O.heat_matrix(mesh, p, phi=phi, u0=u0)
    C = O.heat_matrix(mesh, p, phi=phi, u0=u0, alpha_m=0.0, alpha_k=0.0)
    opc = op.with_alphas(alpha_m=0.0, alpha_k=0.0)
    for M, o in [(A, op), (C, opc)]:
        mf.operator_apply(o, dev(x), y)
        assert relerr(y, M @ x) <= TOL64
        mf.operator_apply_transpose(o, dev(x), y)
        assert relerr(y, M.T @ x) <= TOL64


def test_conv_sine_heaviside_and_velocity_scale(gpu):
    mesh, p, phi, u0 = conv_case((6, 5, 4), W.ALL_FACES, hkind=1, speed=40.0)
    x = W.uniform(1, mesh.n_nodes)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0))
    y = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    A = O.heat_matrix(mesh, p, phi=phi, u0=u0)
    mf.operator_apply(op, dev(x), y)
    assert relerr(y, A @ x) <= TOL64
    mf.operator_apply_transpose(op, dev(x), y)
    assert relerr(y, A.T @ x) <= TOL64


@pytest.mark.parametrize("n,dirichlet", MESHES[1:4])
def test_conv_diagonal(gpu, n, dirichlet):
    mesh, p, phi, u0 = conv_case(n, dirichlet, speed=50.0)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0))
    d = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    for o, kw in [(op, {}), (op.with_alphas(alpha_m=0.0, alpha_k=0.0), {"alpha_m": 0.0, "alpha_k": 0.0})]:
        M = O.heat_matrix(mesh, p, phi=phi, u0=u0, **kw)
        mf.operator_diagonal(o, d)
        assert relerr(d, M.diagonal()) <= TOL64, kw


def test_conv_adjoint_dot_product(gpu):
    # y.(A x) = x.(A^T y) on a mesh too large to assemble quickly
    mesh, p, phi, u0 = conv_case((20, 16, 12), W.FACE_ZLO | W.FACE_XHI, speed=30.0)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0)).with_alphas(alpha_m=0.0, alpha_k=0.0)
    x, yv = dev(W.uniform(2, mesh.n_nodes)), dev(W.uniform(3, mesh.n_nodes))
    ax, aty = torch.empty_like(x), torch.empty_like(x)
    mf.operator_apply(op, x, ax)
    mf.operator_apply_transpose(op, yv, aty)
    lhs, rhs = float(yv @ ax), float(x @ aty)
    assert abs(lhs - rhs) <= 1e-12 * float(yv.abs() @ ax.abs())
    # and the convective part is really not symmetric
    mf.operator_apply(op, yv, aty)
    assert abs(float(x @ aty) - lhs) > 1e-6 * abs(lhs)


def test_conv_full_size(gpu):
    # 64^3 cells (2.15M nodes), the heat benchmark mesh with the Taylor-Green
    # velocity: every entry of A x and A^T x against the assembled oracle matrix
    wl = W.heat_conv_workload(64, W.ALL_FACES)
    nn = wl.mesh.n_nodes
    print("convective heat apply 64^3: assembling the oracle matrix", flush=True)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi, u0=wl.u0)
    x = W.uniform(0, nn)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi), u0=dev(wl.u0))
    y = torch.empty(nn, dtype=torch.float64, device="cuda")
    mf.operator_apply(op, dev(x), y)
    assert relerr(y, O.spmv(A, x)) <= TOL64
    mf.operator_apply_transpose(op, dev(x), y)
    assert relerr(y, A.T @ x) <= TOL64


def test_conv_gmres_jacobi_matches_oracle(gpu):
    # dt = 1e-2: convection is a few percent of the mass term on this mesh
    mesh, p, phi, u0 = conv_case((6, 6, 6), W.ALL_FACES, dt=1e-2)
    A = O.heat_matrix(mesh, p, phi=phi, u0=u0)
    xr = W.uniform(5, mesh.n_nodes)
    b = A @ xr
    dinv = 1.0 / A.diagonal()
    ref = O.gmres(A, b, lambda v: dinv * v, 30, 1e-8)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0))
    x = torch.empty_like(dev(b))
    info = mf.gmres_solve(op, dev(b), x, 1e-8, 500, precond=mf.MF_PC_JACOBI, restart=30)
    print(info, ref.iters, flush=True)
    assert info.converged and abs(info.iters - ref.iters) <= 2
    assert info.rel_res <= 1e-8
    xs = O.direct_solve(A, b)
    info = mf.gmres_solve(op, dev(b), x, 1e-13, 2000, precond=mf.MF_PC_JACOBI, restart=30)
    assert info.converged and relerr(x, xs) <= 1e-10
    # the transposed system
    bt = A.T @ xr
    info = mf.gmres_solve(op, dev(bt), x, 1e-13, 2000, precond=mf.MF_PC_JACOBI, restart=30, transpose=True)
    assert info.converged and relerr(x, O.direct_solve(A.T.tocsr(), bt)) <= 1e-10


@pytest.mark.parametrize("restart", [3, 5])
def test_conv_gmres_short_restarts_match_oracle(gpu, restart):
    # 28-50 restart cycles, each ended by a closing Arnoldi step that only
    # completes the cycle's last Hessenberg column; the oracle takes modified
    # Gram-Schmidt, so the counts agree up to rounding near the threshold
    mesh, p, phi, u0 = conv_case((5, 4, 6), W.ALL_FACES, dt=1e-1)
    A = O.heat_matrix(mesh, p, phi=phi, u0=u0)
    b = A @ W.uniform(11, mesh.n_nodes)
    dinv = 1.0 / A.diagonal()
    ref = O.gmres(A, b, lambda v: dinv * v, restart, 1e-10)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0))
    x = torch.empty_like(dev(b))
    info = mf.gmres_solve(op, dev(b), x, 1e-10, 5000, precond=mf.MF_PC_JACOBI, restart=restart)
    print(info, ref.iters, flush=True)
    assert info.converged and info.rel_res <= 1e-10 and abs(info.iters - ref.iters) <= 3
    # the oracle's own iterate is 7.1e-10 (restart 3) and 7.2e-10 (restart 5) from the direct solution
    xs = O.direct_solve(A, b)
    assert float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs)) <= 1e-8


def test_conv_operator_argument_errors(gpu):
    mesh, p, phi, u0 = conv_case((4, 4, 4), W.ALL_FACES)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi), u0=dev(u0))
    n = mesh.n_nodes
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(mf.MFError, match="symmetric"):  # CG needs a symmetric operator
        mf.cg_solve(op, b, x, 1e-8, 10)
    with pytest.raises(mf.MFError, match="convection"):
        mf.Multigrid(op)
    with pytest.raises(mf.MFError, match="convection"):
        mf.heat_coeff_grad(op, b, b, b, dphi=torch.empty_like(b))
    op32 = mf.heat_operator(ctx, p, phi=dev(phi, torch.float32), u0=dev(u0, torch.float32), precision=mf.MF_FP32)
    with pytest.raises(mf.MFError, match="FP64"):
        mf.operator_apply(op32, b.float(), torch.empty_like(b.float()))
    ones = torch.ones(mesh.n_cells * 27, dtype=torch.float64, device="cuda")
    opq = mf.heat_operator(ctx, p, k_q=ones, rc_q=ones, u0=dev(u0))
    with pytest.raises(mf.MFError, match="LEVELSET"):
        mf.operator_apply(opq, b, x)
