"""GPU interface heat sources (evaporative cooling, laser heat flux) vs the
FP64 oracle, through the C ABI.

Bar (FP64): normwise relative error <= 1e-12 of the right-hand side.  The
kernel and the oracle sum the same products in different orders; the
pointwise terms (square root, exponential, the sine Heaviside) are evaluated
by each side's own math library, within a few ulps.
"""
import dataclasses

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


MESHES = [((1, 1, 1), 0), ((3, 3, 3), W.ALL_FACES), ((5, 3, 7), W.FACE_XLO | W.FACE_ZHI),
          ((9, 9, 9), W.ALL_FACES), ((8, 8, 8), 0), ((17, 10, 5), W.FACE_YHI | W.FACE_XHI)]


def source_case(n, dirichlet, hkind=0, **src):
    wl = W.heat_source_workload(max(n), dirichlet)
    mesh = W.Mesh(n, dirichlet=dirichlet)
    eps = 2.0 / max(n)
    x = W.node_coords(mesh)
    phi = W.phi_sphere(mesh, 0.3, eps)
    T = wl.sources.T_boil + 600.0 * np.exp(-((x[:, 0] - 0.5) ** 2 + (x[:, 1] - 0.5) ** 2) / 0.05) * (x[:, 2] - 0.3)
    p = W.HeatParams(heaviside=hkind, eps=eps if hkind else 0.0)
    # a beam wide enough to reach the sphere's cap on the coarse meshes too
    sp = dataclasses.replace(wl.sources, radius=0.25, **src)
    return mesh, p, sp, phi, T


@pytest.mark.parametrize("n,dirichlet", MESHES)
@pytest.mark.parametrize("terms", [1, 2, 3])
def test_sources_match_oracle(gpu, n, dirichlet, terms):
    mesh, p, sp, phi, T = source_case(n, dirichlet, terms=terms)
    print(f"sources n={n} dirichlet={dirichlet} terms={terms}", flush=True)
    ref = O.heat_sources(mesh, p, sp, phi, T)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi))
    b = torch.full((mesh.n_nodes,), 7.0, dtype=torch.float64, device="cuda")
    mf.heat_source_rhs(op, sp, dev(T), b)
    assert np.abs(ref).max() > 0.0
    assert relerr(b, ref) <= TOL64


@pytest.mark.parametrize("hkind", [0, 1])
def test_sources_heaviside_forms_and_oblique_beam(gpu, hkind):
    # oblique beam off the axis of symmetry, focus away from the centre
    d = np.array([0.3, -0.2, -1.0])
    d /= np.linalg.norm(d)
    mesh, p, sp, phi, T = source_case((7, 6, 8), W.ALL_FACES, hkind=hkind, terms=3, dir=tuple(d),
                                      focus=(0.4, 0.6, 0.9))
    ref = O.heat_sources(mesh, p, sp, phi, T)
    ctx = mf.Context(mesh)
    b = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.heat_source_rhs(mf.heat_operator(ctx, p, phi=dev(phi)), sp, dev(T), b)
    assert relerr(b, ref) <= TOL64


def test_sources_full_size(gpu):
    # 64^3 cells (2.15M nodes), the benchmark workload, every entry against the oracle
    wl = W.heat_source_workload(64, W.ALL_FACES)
    ref = O.heat_sources(wl.mesh, wl.params, wl.sources, wl.phi, wl.T)
    ctx = mf.Context(wl.mesh)
    b = torch.empty(wl.mesh.n_nodes, dtype=torch.float64, device="cuda")
    mf.heat_source_rhs(mf.heat_operator(ctx, wl.params, phi=dev(wl.phi)), wl.sources, dev(wl.T), b)
    assert relerr(b, ref) <= TOL64


def test_sources_argument_errors(gpu):
    mesh, p, sp, phi, T = source_case((4, 4, 4), W.ALL_FACES, terms=3)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(phi))
    b = torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(mf.MFError, match="unit vector"):
        mf.heat_source_rhs(op, dataclasses.replace(sp, dir=(0.0, 0.0, -2.0)), dev(T), b)
    with pytest.raises(mf.MFError, match="temperature"):
        mf.heat_source_rhs(op, sp, None, b)
    with pytest.raises(mf.MFError, match="evaporation"):
        mf.heat_source_rhs(op, dataclasses.replace(sp, evap_coeff=1.5), dev(T), b)
    with pytest.raises(mf.MFError, match="radius"):
        mf.heat_source_rhs(op, dataclasses.replace(sp, radius=0.0), dev(T), b)
    ones = torch.ones(mesh.n_cells * 27, dtype=torch.float64, device="cuda")
    with pytest.raises(mf.MFError, match="LEVELSET"):
        mf.heat_source_rhs(mf.heat_operator(ctx, p, k_q=ones, rc_q=ones), sp, dev(T), b)
    # laser alone needs no temperature
    mf.heat_source_rhs(op, dataclasses.replace(sp, terms=2), None, b)
    ref = O.heat_sources(mesh, p, dataclasses.replace(sp, terms=2), phi, T)
    assert relerr(b, ref) <= TOL64
