"""FP32 geometric multigrid (V-cycle, Chebyshev smoothing, FP64 coarse CG) and
the flexible CG it preconditions, against the FP64 oracle.

Bars:
* lambda_max estimates (FP64 Lanczos on both sides, same start vector and
  step count): relative difference <= 1e-9.
* one V-cycle, same Chebyshev bounds on both sides: GPU FP32 vs oracle FP64
  relative difference <= 2e-6 in the mass-dominated regime (about 30 FP32
  unit roundoffs of 6e-8: rounding enters every apply, transfer and smoother
  update and the degree-4 Chebyshev recurrences amplify it mildly; measured
  6e-8 to 2e-7), 5e-5 where conduction matters (vcycle_bar below).
* flexible CG: the true FP64 residual meets the tolerance, and the solution
  matches the direct solution within kappa * rtol.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2501_18781_amd import mf
from paper_2501_18781_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def relerr(a, b):
    """The larger of the normwise error ||a - b|| / ||b|| and the element-wise
    error max |a - b| / max |b|: a bar on it holds for both."""
    a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else a
    b = np.asarray(b, dtype=np.float64)
    d = np.asarray(a, dtype=np.float64) - b
    return float(max(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300),
                     np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)))


def normerr(a, b):
    """Normwise ||a - b|| / ||b||: the measure of the kappa * rtol bound on the
    solution of a solve stopped at a finite relative residual rtol."""
    a = a.detach().cpu().double().numpy() if isinstance(a, torch.Tensor) else a
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,coarse,dirichlet", [(8, 2, W.ALL_FACES), (16, 4, W.ALL_FACES), (8, 4, 0)])
def test_vcycle_matches_oracle(gpu, n, coarse, dirichlet):
    wl = W.heat_sphere_workload(n, dirichlet)
    print(f"vcycle n={n} coarse={coarse}", flush=True)
    levels = O.heat_mg_levels(wl.mesh, wl.params, wl.phi, n_coarse=coarse)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    lmax = [lv.lmax for lv in levels]
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=coarse, lambda_max=lmax, coarse_rtol=1e-14))
    assert mg.n_levels == len(levels)
    r = W.uniform(3, wl.mesh.n_nodes)
    z = torch.empty_like(dev(r))
    mf.mg_vcycle(mg, dev(r), z)
    ref = O.vcycle(levels, r)
    err = relerr(z, ref)
    print(f"  V-cycle FP32 vs FP64 oracle: {err:.2e}", flush=True)
    assert err <= 2e-6


def test_lanczos_estimates_match_oracle(gpu):
    wl = W.heat_sphere_workload(16, W.ALL_FACES)
    levels = O.heat_mg_levels(wl.mesh, wl.params, wl.phi, n_coarse=4)
    ctx = mf.Context(wl.mesh)
    mg = mf.Multigrid(mf.heat_operator(ctx, wl.params, phi=dev(wl.phi)), mf.MGConfig(coarse_cells=4))
    got = mg.lambda_max()
    for li in range(1, len(levels)):
        assert abs(got[li] - levels[li].lmax) <= 1e-9 * levels[li].lmax, (li, got[li], levels[li].lmax)


def test_flexible_cg_with_multigrid(gpu):
    wl = W.heat_sphere_workload(16, W.ALL_FACES)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    levels = O.heat_mg_levels(wl.mesh, wl.params, wl.phi, n_coarse=4)
    xr = W.uniform(5, wl.mesh.n_nodes)
    b = A @ xr
    ref = O.flexible_cg(A, b, lambda v: O.vcycle(levels, v), rtol=1e-8)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=4, lambda_max=[lv.lmax for lv in levels]))
    x = torch.empty_like(dev(b))
    info = mf.mg_cg_solve(mg, dev(b), x, 1e-8, 100)
    print(info, ref.iters, flush=True)
    assert info.converged and info.rel_res <= 1e-8 and abs(info.iters - ref.iters) <= 1
    assert normerr(x, xr) <= 1e-6
    info = mf.mg_cg_solve(mg, dev(b), x, 1e-13, 100)
    assert info.converged and relerr(x, O.direct_solve(A, b)) <= 1e-11


def test_multigrid_stiff_regime_and_manufactured_rhs(gpu):
    # dt = 100 s at 32^3: k/h^2 exceeds rc/dt in the vapor, the stiffness term
    # dominates and Jacobi-CG needs many more iterations than at dt = 1e-3
    p = W.HeatParams(dt=100.0)
    wl = W.heat_sphere_workload(32, W.ALL_FACES, p)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    b = torch.empty(wl.mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.operator_apply(op, dev(W.manufactured_T(wl.mesh)), b)
    xc, xm = torch.empty_like(b), torch.empty_like(b)
    ic = mf.cg_solve(op, b, xc, 1e-8, 5000)
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=4))
    im = mf.mg_cg_solve(mg, b, xm, 1e-8, 200)
    print(ic, im, flush=True)
    assert ic.converged and im.converged and im.iters < ic.iters / 3
    # both solve the same discrete problem: distance within kappa * rtol
    assert float(torch.linalg.norm(xm - xc) / torch.linalg.norm(xc)) <= 1e-5
    xs = W.manufactured_T(wl.mesh)
    assert float(torch.linalg.norm(xm - dev(xs)) / np.linalg.norm(xs)) <= 1e-5


@pytest.mark.parametrize("dt", [1e-3, 1e3])
def test_multigrid_full_size_128(gpu, dt):
    # The mixed-precision configuration at its full size (128^3 cells,
    # 16,974,593 nodes) and in the launch configuration the benchmark times:
    # properties that hold at any size.  The FCG solution's true residual is
    # within rtol, also at rows the oracle evaluates from its own cell
    # matrices; the FP32 V-cycle is symmetric (to FP32 rounding) and positive.
    p = W.HeatParams(dt=dt)
    wl = W.heat_sphere_workload(128, W.ALL_FACES, p)
    nn = wl.mesh.n_nodes
    print(f"multigrid 128^3 dt={dt}", flush=True)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    b = torch.empty(nn, dtype=torch.float64, device="cuda")
    mf.operator_apply(op, dev(W.manufactured_T(wl.mesh)), b)
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=4))
    try:
        x = torch.empty_like(b)
        info = mf.mg_cg_solve(mg, b, x, 1e-8, 200)
        print(info, mg.n_levels, flush=True)
        assert info.converged and info.rel_res <= 1e-8 and mg.n_levels == 6
        rows = np.unique(np.concatenate([np.random.default_rng(4).integers(0, nn, 200), [0, nn // 2, nn - 1]]))
        bh, xh = b.cpu().numpy(), x.cpu().numpy()
        r_rows = bh[rows] - O.heat_rows(wl.mesh, wl.params, xh, rows, phi=wl.phi)
        assert np.abs(r_rows).max() <= 1e-8 * np.linalg.norm(bh)
        r1, r2 = dev(W.uniform(6, nn)), dev(W.uniform(7, nn))
        z1, z2 = torch.empty_like(r1), torch.empty_like(r1)
        mf.mg_vcycle(mg, r1, z1)
        mf.mg_vcycle(mg, r2, z2)
        a12, a21 = float(r2 @ z1), float(r1 @ z2)
        assert abs(a12 - a21) <= 1e-5 * float(torch.linalg.norm(r2) * torch.linalg.norm(z1))
        assert float(r1 @ z1) > 0.0 and float(r2 @ z2) > 0.0
    finally:
        mg.close()


def test_multigrid_argument_errors(gpu):
    wl = W.heat_sphere_workload(10, W.ALL_FACES)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    with pytest.raises(mf.MFError):
        mf.Multigrid(op, mf.MGConfig(coarse_cells=2))  # 10 -> 5 cannot halve again
    with pytest.raises(mf.MFError):
        mf.Multigrid(op, mf.MGConfig(coarse_cells=16))  # already coarse
    assert mf.Multigrid(op, mf.MGConfig(coarse_cells=5)).n_levels == 2
    kq = torch.ones(ctx.n_cells * 27, dtype=torch.float64, device="cuda")
    with pytest.raises(mf.MFError):
        mf.Multigrid(mf.heat_operator(ctx, wl.params, k_q=kq, rc_q=kq), mf.MGConfig(coarse_cells=3))


def oracle_hierarchy_like(wl, mg):
    """The oracle's levels with the GPU hierarchy's sizes and Chebyshev bounds,
    and its coarsest-level treatment: Chebyshev smoothing from zero with the
    same degree and bounds, or (degree 0) the exact solve."""
    info = mg.levels()  # (cells, degree, lambda_min, lambda_max), coarsest first
    cells0, deg0, lmin0, lmax0 = info[0]
    levels = O.heat_mg_levels(wl.mesh, wl.params, wl.phi, n_coarse=cells0, lmax_override=[lv[3] for lv in info])
    assert len(levels) == len(info)
    coarse = None
    if deg0 > 0:
        L0 = levels[0]
        coarse = lambda v: O.chebyshev_smooth(lambda u: O.spmv(L0.A, u), L0.dinv, v, None, deg0, lmin0, lmax0)
    return levels, coarse


# FP32 V-cycle against the FP64 oracle where conduction matters: the FP32
# rounding of the sum-factorized contractions is relative to the largest
# terms of a cell, the liquid's, while the gas conducts 100 times less
# (k 30 / 0.3), so the gas-side result carries about 100 u32 = 6e-6 per
# operator application; a few dependent applications per V-cycle give the bar
# 5e-5 (measured 1.4e-5 at 32^3, dt = 1).  Mass-dominated (dt = 1e-3): 2e-6.
def vcycle_bar(dt):
    return 2e-6 if dt <= 1e-3 else 5e-5


@pytest.mark.parametrize("dt", [1.0, 1e3])
def test_vcycle_matches_oracle_where_conduction_matters(gpu, dt):
    wl = W.heat_sphere_workload(16, W.ALL_FACES, W.HeatParams(dt=dt))
    levels = O.heat_mg_levels(wl.mesh, wl.params, wl.phi, n_coarse=4)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=4, lambda_max=[lv.lmax for lv in levels], coarse_rtol=1e-14))
    r = W.uniform(3, wl.mesh.n_nodes)
    z = torch.empty_like(dev(r))
    mf.mg_vcycle(mg, dev(r), z)
    err = relerr(z, O.vcycle(levels, r))
    print(f"V-cycle dt={dt}: {err:.2e}", flush=True)
    assert err <= vcycle_bar(dt)


# The level rule: the first level from the finest down with
# beta = 17.5 * 3 / h^2 * max(k / rc) * dt <= 1 is smoothed, not solved.
# Here max(k / rc) = 0.3 / 5e3 (the gas): beta = 3.15e-3 n^2 dt.
#   16^3, dt = 1e-3: beta = 8e-4          -> one level, smoothed
#   32^3, dt = 1:    3.2 (32^3), 0.81 (16^3) -> 32^3 and a smoothed 16^3
#   16^3, dt = 1e3:  806, 201, 50, 12.6    -> down to 2^3, solved by CG
@pytest.mark.parametrize("n,dt,nlev,coarsest_degree", [(16, 1e-3, 1, 2), (32, 1.0, 2, 2), (16, 1e3, 4, 0)])
def test_level_rule_vcycle_and_flexible_cg(gpu, n, dt, nlev, coarsest_degree):
    wl = W.heat_sphere_workload(n, W.ALL_FACES, W.HeatParams(dt=dt))
    print(f"level rule n={n} dt={dt}", flush=True)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=2, degree=4, auto_levels=True, smooth_degree=2))
    info = mg.levels()
    print(info, flush=True)
    assert mg.n_levels == nlev and info[-1][0] == n and info[0][1] == coarsest_degree
    if coarsest_degree:  # bounds of the smoothed level bracket the Lanczos estimate of its spectrum
        assert 0.0 < info[0][2] < info[0][3]
    levels, coarse = oracle_hierarchy_like(wl, mg)
    r = W.uniform(3, wl.mesh.n_nodes)
    z = torch.empty_like(dev(r))
    mf.mg_vcycle(mg, dev(r), z)
    err = relerr(z, O.vcycle(levels, r, degree=4, coarse_solve=coarse))
    print(f"  V-cycle FP32 vs FP64 oracle: {err:.2e}", flush=True)
    assert err <= vcycle_bar(dt)
    A = levels[-1].A
    xr = W.uniform(5, wl.mesh.n_nodes)
    b = A @ xr
    ref = O.flexible_cg(A, b, lambda v: O.vcycle(levels, v, degree=4, coarse_solve=coarse), rtol=1e-8)
    x = torch.empty_like(dev(b))
    res = mf.mg_cg_solve(mg, dev(b), x, 1e-8, 200)
    print(res, ref.iters, flush=True)
    assert res.converged and res.rel_res <= 1e-8 and abs(res.iters - ref.iters) <= 1
    assert normerr(x, xr) <= 1e-6


def test_flexible_cg_at_scale_matches_oracle_and_repeats_bitwise(gpu):
    # The benchmark's hierarchy in the conduction-dominated regime on 64^3
    # cells (five V-cycle levels of Chebyshev(1), 4^3 by FP64 CG): the GPU
    # flexible CG takes the oracle's iteration count (its V-cycle in FP64 with
    # the same bounds) within one, and three solves give bitwise the same
    # iterate.  Every scalar of the iteration (alpha, beta, the convergence
    # test) is formed on the device by launches whose workgroups all read the
    # same inputs; a workgroup that saw another's update of a scalar it reads
    # would change the direction of part of the vector, and the iteration
    # count and bits with it.
    wl = W.heat_sphere_workload(64, W.ALL_FACES, W.HeatParams(dt=1e3))
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=4, degree=1, auto_levels=True, smooth_degree=2))
    info = mg.levels()
    assert [lv[0] for lv in info] == [4, 8, 16, 32, 64] and all(lv[1] == 1 for lv in info[1:])
    b = dev(W.uniform(5, wl.mesh.n_nodes))
    xs, its = [], []
    for _ in range(3):
        x = torch.empty_like(b)
        res = mf.mg_cg_solve(mg, b, x, 1e-8, 200)
        assert res.converged and res.rel_res <= 1e-8
        xs.append(x.cpu().numpy())
        its.append(res.iters)
    print("GPU FCG iterations", its, flush=True)
    assert its[0] == its[1] == its[2]
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    levels, coarse = oracle_hierarchy_like(wl, mg)
    print("oracle flexible CG at 64^3", flush=True)
    ref = O.flexible_cg(levels[-1].A, b.cpu().numpy(), lambda v: O.vcycle(levels, v, degree=1, coarse_solve=coarse),
                        rtol=1e-8)
    print(its[0], ref.iters, flush=True)
    assert abs(its[0] - ref.iters) <= 1


def test_flexible_cg_edge_cases(gpu):
    # a zero right-hand side and maxit = 0 stop before the first iteration
    # with x = 0 (the first V-cycle runs without a poll before it, on a solve
    # that is already done); a small maxit is reported with that many
    # iterations done
    wl = W.heat_sphere_workload(8, W.ALL_FACES)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    mg = mf.Multigrid(op, mf.MGConfig(coarse_cells=4))
    n = wl.mesh.n_nodes
    x = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    info = mf.mg_cg_solve(mg, torch.zeros(n, dtype=torch.float64, device="cuda"), x, 1e-8, 50)
    assert info.converged and info.iters == 0 and float(x.abs().max()) == 0.0
    b = dev(W.uniform(3, n))
    x.fill_(7.0)
    info = mf.mg_cg_solve(mg, b, x, 1e-8, 0)
    assert info.status == mf.MF_NOT_CONVERGED and info.iters == 0 and float(x.abs().max()) == 0.0
    info = mf.mg_cg_solve(mg, b, x, 1e-14, 2)
    assert info.status == mf.MF_NOT_CONVERGED and info.iters == 2
