"""GPU heat operator vs the FP64 oracle, through the C ABI.

Bar (FP64): normwise relative error <= 1e-12 for applies and diagonals.  The
FP32 apply is held to 2e-6: about 27 rounded terms of unit roundoff 6e-8 per
output, accumulated through three contraction passes each way.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2501_18781_amd import mf
from paper_2501_18781_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-6


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


def normerr(a, b):
    """Normwise ||a - b|| / ||b||: the measure of the kappa * rtol bound on the
    solution of a solve stopped at a finite relative residual rtol."""
    a = a.detach().cpu().double().numpy() if isinstance(a, torch.Tensor) else a
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def heat_case(n, dirichlet, seed=0, phi_kind="sphere", hkind=0):
    mesh = W.Mesh(n, dirichlet=dirichlet)
    eps = 2.0 / max(n)
    if phi_kind == "sphere":
        phi = W.phi_sphere(mesh, 0.3, eps)
    else:  # overshooting random field: exercises the clamp of H
        phi = 1.5 * W.uniform(seed + 100, mesh.n_nodes)
    p = W.HeatParams(heaviside=hkind, eps=eps if hkind else 0.0)
    return mesh, p, phi


# meshes smaller than, equal to and straddling the 4x4x4-cell brick, with ragged tails
MESHES = [((1, 1, 1), 0), ((3, 3, 3), W.ALL_FACES), ((5, 3, 7), W.FACE_XLO | W.FACE_ZHI),
          ((9, 9, 9), W.ALL_FACES), ((8, 8, 8), 0), ((17, 10, 5), W.FACE_YHI | W.FACE_XHI)]


@pytest.mark.parametrize("n,dirichlet", MESHES)
def test_heat_apply_fp64_matches_oracle(gpu, n, dirichlet):
    mesh, p, phi = heat_case(n, dirichlet)
    print(f"heat apply fp64 n={n} dirichlet={dirichlet}", flush=True)
    A = O.heat_matrix(mesh, p, phi=phi)
    x = W.uniform(0, mesh.n_nodes)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi))
    y = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_apply(op, dev(x), y)
    assert relerr(y, A @ x) <= TOL64
    # each term on its own: the stiffness part is ~1e-5 of the total here
    for am, ak in [(0.0, 1.0), (1.0, 0.0)]:
        Ai = O.heat_matrix(mesh, p, phi=phi, alpha_m=am * p.alpha_m, alpha_k=ak)
        mf.operator_apply(op.with_alphas(alpha_m=am * p.alpha_m, alpha_k=ak), dev(x), y)
        assert relerr(y, Ai @ x) <= TOL64, (am, ak)
    # transpose of the symmetric operator is the same map
    yt = torch.empty_like(y)
    mf.operator_apply_transpose(op, dev(x), yt)
    assert relerr(yt, A @ x) <= TOL64


@pytest.mark.parametrize("hkind,phi_kind", [(0, "random"), (1, "sphere"), (1, "random")])
def test_heat_apply_heaviside_forms(gpu, hkind, phi_kind):
    mesh, p, phi = heat_case((6, 5, 4), W.ALL_FACES, phi_kind=phi_kind, hkind=hkind)
    if phi_kind == "random":
        phi = np.clip(phi, -0.999, 0.999) if hkind else phi
    A = O.heat_matrix(mesh, p, phi=phi)
    x = W.uniform(1, mesh.n_nodes)
    ctx = mf.Context(mesh)
    y = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_apply(mf.heat_operator(ctx, p, phi=dev(phi)), dev(x), y)
    assert relerr(y, A @ x) <= TOL64


# (7, 4, 5) cells on the unit cube have unequal edges, (6, 6, 6) equal ones:
# the two forms of the derivative passes
@pytest.mark.parametrize("n", [(7, 4, 5), (6, 6, 6)])
def test_heat_apply_quadrature_point_coefficients(gpu, n):
    mesh = W.Mesh(n, dirichlet=W.FACE_ZLO | W.FACE_YHI)
    print(f"heat apply, coefficients per quadrature point, n={n}", flush=True)
    rng = np.random.default_rng(5)
    kq = rng.uniform(0.3, 30.0, mesh.n_cells * 27)
    rcq = rng.uniform(5e3, 5e6, mesh.n_cells * 27)
    p = W.HeatParams()
    A = O.heat_matrix(mesh, p, kq=kq, rcq=rcq)
    x = W.uniform(2, mesh.n_nodes)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, k_q=dev(kq), rc_q=dev(rcq))
    y = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_apply(op, dev(x), y)
    assert relerr(y, A @ x) <= TOL64
    Ak = O.heat_matrix(mesh, p, kq=kq, rcq=rcq, alpha_m=0.0)
    mf.operator_apply(op.with_alphas(alpha_m=0.0), dev(x), y)
    assert relerr(y, Ak @ x) <= TOL64


def test_heat_apply_anisotropic_box(gpu):
    mesh = W.Mesh((4, 6, 3), lo=(-0.5, 0.0, 1.0), hi=(1.5, 0.6, 1.3), dirichlet=W.FACE_XHI)
    phi = 0.8 * W.uniform(9, mesh.n_nodes)
    p = W.HeatParams()
    A = O.heat_matrix(mesh, p, phi=phi, alpha_m=1.0)
    x = W.uniform(3, mesh.n_nodes)
    ctx = mf.Context(mesh)
    y = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_apply(mf.heat_operator(ctx, p, phi=dev(phi), alpha_m=1.0), dev(x), y)
    assert relerr(y, A @ x) <= TOL64


@pytest.mark.parametrize("n,dirichlet", MESHES[:4])
def test_heat_apply_fp32(gpu, n, dirichlet):
    mesh, p, phi = heat_case(n, dirichlet)
    A = O.heat_matrix(mesh, p, phi=phi.astype(np.float32).astype(np.float64))
    x = W.uniform(0, mesh.n_nodes).astype(np.float32)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi, torch.float32), precision=mf.MF_FP32)
    y = torch.empty(mesh.n_nodes, dtype=torch.float32, device="cuda")
    mf.operator_apply(op, dev(x, torch.float32), y)
    assert relerr(y, A @ x.astype(np.float64)) <= TOL32


# Meshes around the 4x4x8-cell bricks of the FP32 applies: exactly one brick,
# ragged z tails, several bricks along z, equal and unequal cell edges.
DEEP = [((4, 4, 8), W.ALL_FACES), ((3, 2, 9), 0), ((6, 5, 19), W.FACE_ZLO | W.FACE_YHI),
        ((12, 12, 12), W.FACE_YLO | W.FACE_ZHI), ((5, 9, 17), W.FACE_XHI)]


@pytest.mark.parametrize("hkind", [0, 1])
@pytest.mark.parametrize("n,dirichlet", DEEP)
def test_heat_apply_fp32_deep_bricks(gpu, n, dirichlet, hkind):
    mesh, p, phi = heat_case(n, dirichlet, hkind=hkind)
    print(f"heat apply fp32 n={n} dirichlet={dirichlet} hkind={hkind}", flush=True)
    phi32 = phi.astype(np.float32)
    A = O.heat_matrix(mesh, p, phi=phi32.astype(np.float64))
    x = W.uniform(4, mesh.n_nodes).astype(np.float32)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi32, torch.float32), precision=mf.MF_FP32)
    y = torch.empty(mesh.n_nodes, dtype=torch.float32, device="cuda")
    mf.operator_apply(op, dev(x, torch.float32), y)
    assert relerr(y, A @ x.astype(np.float64)) <= TOL32


@pytest.mark.parametrize("n", [(6, 6, 6), (7, 4, 13)])
def test_heat_apply_fp32_quadrature_point_coefficients(gpu, n):
    mesh = W.Mesh(n, dirichlet=W.FACE_ZLO | W.FACE_XHI)
    print(f"heat apply fp32, coefficients per quadrature point, n={n}", flush=True)
    rng = np.random.default_rng(6)
    kq = rng.uniform(0.3, 30.0, mesh.n_cells * 27).astype(np.float32)
    rcq = rng.uniform(5e3, 5e6, mesh.n_cells * 27).astype(np.float32)
    p = W.HeatParams()
    x = W.uniform(5, mesh.n_nodes).astype(np.float32)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, k_q=dev(kq, torch.float32), rc_q=dev(rcq, torch.float32), precision=mf.MF_FP32)
    y = torch.empty(mesh.n_nodes, dtype=torch.float32, device="cuda")
    for am in (p.alpha_m, 0.0):  # the whole operator, then the stiffness part alone
        A = O.heat_matrix(mesh, p, kq=kq.astype(np.float64), rcq=rcq.astype(np.float64), alpha_m=am)
        mf.operator_apply(op.with_alphas(alpha_m=am), dev(x, torch.float32), y)
        assert relerr(y, A @ x.astype(np.float64)) <= TOL32, am


@pytest.mark.parametrize("n,dirichlet", MESHES[1:4])
def test_heat_diagonal(gpu, n, dirichlet):
    mesh, p, phi = heat_case(n, dirichlet)
    A = O.heat_matrix(mesh, p, phi=phi)
    ctx = mf.Context(mesh)
    d = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_diagonal(mf.heat_operator(ctx, p, phi=dev(phi)), d)
    assert relerr(d, A.diagonal()) <= TOL64


def test_heat_apply_full_size(gpu):
    # 64^3 cells (2,146,689 nodes), the benchmark configuration: every entry
    # of y = A x and of the stiffness part alone against the oracle's
    # assembled matrix (1.35e8 nonzeros)
    n = 64
    wl = W.heat_sphere_workload(n, W.ALL_FACES)
    print("heat apply 64^3: assembling the oracle matrix", flush=True)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    x = W.uniform(0, wl.mesh.n_nodes)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    y = torch.empty(wl.mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_apply(op, dev(x), y)
    assert relerr(y, O.spmv(A, x)) <= TOL64
    del A
    K = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi, alpha_m=0.0)
    mf.operator_apply(op.with_alphas(alpha_m=0.0), dev(x), y)
    assert relerr(y, O.spmv(K, x)) <= TOL64


def test_cg_jacobi_matches_oracle_iterations_and_solution(gpu):
    # 8^3 cells, no Dirichlet, b = A x_ref, Jacobi-CG to 1e-10
    wl = W.heat_sphere_workload(8, 0)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    xr = W.uniform(0, wl.mesh.n_nodes)
    b = A @ xr
    ref = O.jacobi_cg(A, b, 1e-10)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    x = torch.empty_like(dev(b))
    info = mf.cg_solve(op, dev(b), x, 1e-10, 1000)
    print(info, ref.iters, flush=True)
    assert info.converged and abs(info.iters - ref.iters) <= 1
    assert info.rel_res <= 1e-10 * 1.5
    # the iterates agree with the oracle's CG to within the rounding of the recurrences
    assert normerr(x, ref.x) <= 1e-9
    # tight tolerance: the discrete solution itself
    xs = O.direct_solve(A, b)
    info = mf.cg_solve(op, dev(b), x, 1e-14, 1000)
    assert relerr(x, xs) <= 1e-12


@pytest.mark.parametrize("n,dirichlet", [((5, 6, 7), W.ALL_FACES), ((9, 3, 4), W.FACE_XLO)])
def test_cg_ragged_meshes(gpu, n, dirichlet):
    mesh, p, phi = heat_case(n, dirichlet)
    A = O.heat_matrix(mesh, p, phi=phi)
    b = A @ W.uniform(4, mesh.n_nodes)
    ref = O.jacobi_cg(A, b, 1e-10)
    ctx = mf.Context(mesh)
    x = torch.empty_like(dev(b))
    info = mf.cg_solve(mf.heat_operator(ctx, p, phi=dev(phi)), dev(b), x, 1e-10, 1000)
    assert info.converged and abs(info.iters - ref.iters) <= 1
    assert normerr(x, O.direct_solve(A, b)) <= 1e-9


def test_cg_edge_cases(gpu):
    wl = W.heat_sphere_workload(3, W.ALL_FACES)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    n = wl.mesh.n_nodes
    x = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    info = mf.cg_solve(op, torch.zeros(n, dtype=torch.float64, device="cuda"), x, 1e-10, 100)
    assert info.converged and info.iters == 0 and float(x.abs().max()) == 0.0
    # maxit reached: status reported, x holds the last iterate
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    b = A @ W.uniform(0, n)
    info = mf.cg_solve(op, dev(b), x, 1e-14, 2)
    assert info.status == mf.MF_NOT_CONVERGED and info.iters == 2
    # iteration limits at and just past the first poll (after 8 iterations,
    # with one more already queued behind it) stop exactly there
    for maxit in (8, 9, 10):
        info = mf.cg_solve(op, dev(b), x, 1e-30, maxit)
        assert info.status == mf.MF_NOT_CONVERGED and info.iters == maxit, maxit
    # an indefinite operator (negative mass factor) is reported as a breakdown
    bad = op.with_alphas(alpha_m=-1e3, alpha_k=0.0)
    info = mf.cg_solve(bad, dev(b), x, 1e-10, 100, precond=mf.MF_PC_NONE)
    assert info.status == mf.MF_BREAKDOWN
    with pytest.raises(mf.MFError):
        mf.cg_solve(op, dev(b), x, 1e-10, 100, precond=mf.MF_PC_BLOCK_JACOBI)


def test_heat_apply_largest_mesh(gpu):
    # the largest cube the boundary accepts: 446^3 cells, 893^3 = 712,121,957
    # nodes (3 n_nodes < 2^31), 5.7 GB per nodal vector; sampled rows against
    # the oracle's cell matrices, including the first and last node
    mesh = W.Mesh((446, 446, 446), dirichlet=W.ALL_FACES)
    nn = mesh.n_nodes
    assert 3 * nn < 2 ** 31
    print(f"largest mesh: {nn} nodes", flush=True)
    p = W.HeatParams()
    phi = W.phi_sphere(mesh, 0.3, 2.0 / 446)
    x = W.uniform(0, nn)
    print("inputs ready", flush=True)
    ctx = mf.Context(mesh)
    xd = dev(x)
    y = torch.empty(nn, dtype=torch.float64, device="cuda")
    mf.operator_apply(mf.heat_operator(ctx, p, phi=dev(phi)), xd, y)
    rows = np.unique(np.concatenate([np.random.default_rng(12).integers(0, nn, 300), [0, 1, nn // 2, nn - 1]]))
    got = y[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    ref = O.heat_rows(mesh, p, x, rows, phi=phi)
    assert np.abs(got - ref).max() <= TOL64 * np.abs(ref).max()
