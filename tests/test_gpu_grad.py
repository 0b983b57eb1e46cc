"""Gradients of a temperature misfit through one implicit heat step: the GPU
adjoint (hand-written gradient kernel + adjoint CG, via torch.autograd)
against the oracle's assembled-matrix adjoint and against central finite
differences.

Loss: L = sum_i (dT_i - dT_tgt,i)^2 with dT = T - T_old (delta form, same
minimizer as ||T - T_tgt||^2 since T_old is fixed).  The target comes from
the conductivity k(1 + 0.1 sin(2 pi x)) at the quadrature points.
Bars, each both normwise and element-wise (max |a - ref| <= tol max |ref|):
kernel parity 1e-12; adjoint gradients vs the oracle 1e-9 (both sides solve
to rtol 1e-14, kappa ~ 16); finite differences 1e-6 (see below).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2501_18781_amd import mf
from paper_2501_18781_amd import workloads as W
from paper_2501_18781_amd.autograd import HeatStep, heat_step

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    """The larger of the normwise error ||a - b|| / ||b|| and the element-wise
    error max |a - b| / max |b|: a bar on it holds for both."""
    a = host(a) if isinstance(a, torch.Tensor) else a
    b = np.asarray(b, dtype=np.float64)
    d = np.asarray(a, dtype=np.float64) - b
    return float(max(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300),
                     np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)))


def close(a, b, tol):
    """Normwise and element-wise agreement within tol (relative to the reference's size)."""
    a = host(a) if isinstance(a, torch.Tensor) else a
    return relerr(a, b) <= tol and np.abs(a - b).max() <= tol * np.abs(b).max()


def boundary_mask(mesh):
    x = W.node_coords(mesh)
    return np.any((x == 0.0) | (x == 1.0), axis=1)


def t_old(mesh):
    T = W.manufactured_T(mesh)
    T[boundary_mask(mesh)] = 0.0  # homogeneous Dirichlet on all faces
    return T


@pytest.mark.parametrize("hkind", [0, 1])
def test_gradient_kernel_matches_oracle(gpu, hkind):
    p = W.HeatParams(heaviside=hkind, eps=2.0 / 5 if hkind else 0.0)
    wl = W.heat_sphere_workload(5, W.ALL_FACES, p)
    nn = wl.mesh.n_nodes
    T, dT, lam = W.uniform(1, nn), 1e-3 * W.uniform(2, nn), W.uniform(3, nn)
    dk_ref, drc_ref, dphi_ref = O.heat_grad(wl.mesh, wl.params, T, T - dT, lam, phi=wl.phi, dT=dT)
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    nq = ctx.n_cells * 27
    dk = torch.empty(nq, dtype=torch.float64, device="cuda")
    drc = torch.empty_like(dk)
    dphi = torch.empty(nn, dtype=torch.float64, device="cuda")
    mf.heat_coeff_grad(op, dev(T), dev(dT), dev(lam), dk, drc, dphi)
    assert close(dk, dk_ref, 1e-12)
    assert close(drc, drc_ref, 1e-12)
    assert close(dphi, dphi_ref, 1e-12)


def oracle_grad(mesh, p, phi, kq, rcq, Told, dTt, wrt_phi):
    """Assembled adjoint: dT from the delta form, lam from A^T lam = 2 (dT - dT_tgt) on free nodes."""
    A = O.heat_matrix(mesh, p, kq=kq, rcq=rcq)
    K = O.heat_matrix(mesh, p, kq=kq, rcq=rcq, alpha_m=0.0)
    free = ~O.constrained_mask(mesh)
    r = -(K @ Told) * free
    dT = O.jacobi_cg(A, r, 1e-14).x
    g = 2 * (dT - dTt) * free
    lam = O.jacobi_cg(A.T.tocsr(), g, 1e-14).x
    dk, drc, dphi = O.heat_grad(mesh, p, Told + dT, Told, lam, phi=phi if wrt_phi else None, dT=dT)
    return dT, dk, drc, dphi


def target_delta(mesh, p, phi, kq, rcq, xq, Told):
    kt = kq * (1.0 + 0.1 * np.sin(2 * np.pi * xq[:, 0]))
    A = O.heat_matrix(mesh, p, kq=kt, rcq=rcq)
    K = O.heat_matrix(mesh, p, kq=kt, rcq=rcq, alpha_m=0.0)
    free = ~O.constrained_mask(mesh)
    return O.jacobi_cg(A, -(K @ Told) * free, 1e-14).x


# 32^3 cells (274,625 nodes, 884,736 quadrature points) is the differentiation
# configuration, with the linear Heaviside H = (1 + phi)/2
@pytest.mark.parametrize("n", [4, 8, 32])
def test_autograd_step_matches_oracle_adjoint(gpu, n):
    print(f"autograd vs oracle adjoint, {n}^3 cells", flush=True)
    wl = W.heat_sphere_workload(n, W.ALL_FACES)
    assert wl.params.heaviside == mf.MF_H_LINEAR
    mesh, p = wl.mesh, wl.params
    Told = t_old(mesh)
    # oracle side, its own coefficients, quadrature points and target
    kq, rcq = O.heat_qp_coeffs(mesh, p, wl.phi)
    dTt = target_delta(mesh, p, wl.phi, kq, rcq, O.quad_points(mesh), Told)
    dT_ref, dk_ref, drc_ref, _ = oracle_grad(mesh, p, wl.phi, kq, rcq, Told, dTt, False)
    _, _, _, dphi_ref = oracle_grad(mesh, p, wl.phi, kq, rcq, Told, dTt, True)
    # GPU side: coefficients at quadrature points from the library itself
    ctx = mf.Context(mesh)
    step = HeatStep(ctx, p)
    kq_g = torch.empty(ctx.n_cells * 27, dtype=torch.float64, device="cuda")
    rcq_g = torch.empty_like(kq_g)
    mf.heat_qp_coeffs(step.operator(phi=dev(wl.phi)), kq_g, rcq_g)
    assert close(kq_g, kq, 1e-14) and close(rcq_g, rcq, 1e-14)
    kq_g.requires_grad_(True)
    rcq_g.requires_grad_(True)
    _, dT = heat_step(step, dev(Told), k_q=kq_g, rc_q=rcq_g)
    assert close(dT, dT_ref, 1e-11)
    L = torch.sum((dT - dev(dTt)) ** 2)
    L.backward()
    assert close(kq_g.grad, dk_ref, 1e-9)
    assert close(rcq_g.grad, drc_ref, 1e-9)
    phi = dev(wl.phi).requires_grad_(True)
    _, dT2 = heat_step(step, dev(Told), phi=phi)
    torch.sum((dT2 - dev(dTt)) ** 2).backward()
    assert close(phi.grad, dphi_ref, 1e-9)


def test_finite_differences_32(gpu):
    """Heat step at 32^3 cells, 20 random directions per parameter group (k and
    rc multiplicative, phi additive), directions from numpy's generator with
    seed 2 drawn in the order k, rc, phi.  Two difference formulas:

    * central, step 1e-6: truncation s^2 f^(3) / 6; along phi the loss varies
      on the scale of the interface band (central differences at s = 1e-4 err
      by 8.6e-4 there), which gives about 1e-7 at s = 1e-6; rounding: the loss
      carries a relative error below about 4e-13 from the rtol 1e-14 solves,
      divided by s gives about 4e-7.  Bar: 1e-6 (measured worst 8.6e-8).
    * fourth-order five-point, step 5e-5: truncation s^4 f^(5) / 30, about
      6e-8 along phi; rounding about 1.5 * 4e-13 / s = 1.2e-8.  Bar: 1e-6
      (measured worst: 2e-9 for k, 1e-9 for rc, 1.1e-8 for phi).

    Uses the sine Heaviside, which is twice continuously differentiable in phi.
    The clamped linear form has kinks at phi_q = +-1, which the Q2 interpolant
    of the tanh profile reaches where it overshoots; the loss is not
    differentiable there, so that form's phi gradient is checked only against
    the oracle's assembled adjoint."""
    n = 32
    wl = W.heat_sphere_workload(n, W.ALL_FACES, W.HeatParams(heaviside=1, eps=2.0 / n))
    mesh, p = wl.mesh, wl.params
    ctx = mf.Context(mesh)
    step = HeatStep(ctx, p)
    Told = dev(t_old(mesh))
    phi0 = dev(wl.phi)
    nq = ctx.n_cells * 27
    kq = torch.empty(nq, dtype=torch.float64, device="cuda")
    rcq = torch.empty_like(kq)
    mf.heat_qp_coeffs(step.operator(phi=phi0), kq, rcq)
    xq = torch.empty(nq * 3, dtype=torch.float64, device="cuda")
    mf.quad_points(ctx, xq)
    kt = kq * (1.0 + 0.1 * torch.sin(2 * np.pi * xq.view(-1, 3)[:, 0]))
    _, dTt = heat_step(step, Told, k_q=kt, rc_q=rcq)
    dTt = dTt.detach()

    def loss(k=None, rc=None, phi=None):
        if phi is not None:
            _, dT = heat_step(step, Told, phi=phi)
        else:
            _, dT = heat_step(step, Told, k_q=k, rc_q=rc)
        return float(torch.sum((dT - dTt) ** 2))

    kg, rg = kq.clone().requires_grad_(True), rcq.clone().requires_grad_(True)
    torch.sum((heat_step(step, Told, k_q=kg, rc_q=rg)[1] - dTt) ** 2).backward()
    pg = phi0.clone().requires_grad_(True)
    torch.sum((heat_step(step, Told, phi=pg)[1] - dTt) ** 2).backward()
    rng = np.random.default_rng(2)
    dirs = {g: [dev(rng.uniform(-1, 1, nq if g != "phi" else mesh.n_nodes)) for _ in range(20)]
            for g in ("k", "rc", "phi")}
    def central(f, s=1e-6):
        return (f(s) - f(-s)) / (2 * s)

    def five_point(f, s=5e-5):
        return (8 * (f(s) - f(-s)) - (f(2 * s) - f(-2 * s))) / (12 * s)

    worst = {"central": {}, "five_point": {}}
    with torch.no_grad():
        for g, v in [(g, v) for g in ("k", "rc", "phi") for v in dirs[g]]:
            if g == "k":
                f = lambda t: loss(k=kq * (1 + t * v), rc=rcq)
                ad = float(torch.sum(kg.grad * kq * v))
            elif g == "rc":
                f = lambda t: loss(k=kq, rc=rcq * (1 + t * v))
                ad = float(torch.sum(rg.grad * rcq * v))
            else:
                f = lambda t: loss(phi=phi0 + t * v)
                ad = float(torch.sum(pg.grad * v))
            for name, rule in (("central", central), ("five_point", five_point)):
                e = abs(rule(f) - ad) / abs(ad)
                worst[name][g] = max(worst[name].get(g, 0.0), e)
    for name, w in worst.items():
        print(f"worst relative FD mismatch, {name} (20 directions per group):",
              {g: f"{e:.2e}" for g, e in w.items()}, flush=True)
    assert max(worst["central"].values()) <= 1e-6
    assert max(worst["five_point"].values()) <= 1e-6


def test_heat_step_holds_boundary_values(gpu):
    # T_old nonzero on the Dirichlet faces: the walls keep T_old and the free
    # rows see it (the lifted step of the oracle, in delta form)
    wl = W.heat_sphere_workload(8, W.ALL_FACES)
    mesh, n = wl.mesh, wl.mesh.n_nodes
    Told = 2000.0 + 300.0 * W.manufactured_T(mesh) + 10.0 * W.uniform(6, n)
    T_ref, dT_ref = O.heat_step(mesh, wl.params, Told, phi=wl.phi, delta=True)
    ctx = mf.Context(mesh)
    step = HeatStep(ctx, wl.params)
    T, dT = heat_step(step, dev(Told), phi=dev(wl.phi))
    assert close(dT, dT_ref, 1e-11)
    cm = O.constrained_mask(mesh)
    assert np.array_equal(host(T)[cm], Told[cm]) and not host(dT)[cm].any()
    assert np.abs(host(T) - T_ref).max() <= 1e-14 * np.abs(T_ref).max()


def test_gradient_wrt_t_old_by_brute_force_jacobian(gpu):
    # The step is linear in T_old: T = T_old + dT with dT = J T_old, where J
    # is formed column by column from the oracle's step on unit vectors (343
    # nodes).  For L = w1.T + w2.dT, dL/dT_old = w1 + J^T (w1 + w2); the part
    # J^T (w1 + w2), about 1e-5 of w1 at this time step, is compared on its own.
    wl = W.heat_sphere_workload(3, W.ALL_FACES)
    mesh, n = wl.mesh, wl.mesh.n_nodes
    J = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        J[:, j] = O.heat_step(mesh, wl.params, e, phi=wl.phi, delta=True)[1]
    w1, w2 = W.uniform(9, n), 1e3 * W.uniform(10, n)
    ref = J.T @ (w1 + w2)
    ctx = mf.Context(mesh)
    step = HeatStep(ctx, wl.params)
    Told = dev(500.0 + 100.0 * W.uniform(11, n)).requires_grad_(True)
    T, dT = heat_step(step, Told, phi=dev(wl.phi))
    (torch.sum(T * dev(w1)) + torch.sum(dT * dev(w2))).backward()
    g = host(Told.grad)
    assert close(g - w1, ref, 1e-9)
    assert close(g, w1 + ref, 1e-13)
