"""The allocation-free apply (mf_operator_apply_noalloc) against the
allocating one (mf_operator_apply), through the C ABI: two calls in a row on
one GPU, the second on a smaller mesh (the fixed scratch array keeps the first
call's contents), for the heat operator in FP64 and FP32 and the Oseen
operator.  Bar: 1e-12 (FP64) / 2e-6 (FP32) against the other entry point,
normwise and element-wise; both run the same kernels, so the results are in
fact bitwise equal, which is checked too."""
import numpy as np
import pytest
import torch

from paper_2501_18781_amd import mf
from paper_2501_18781_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def relerr(a, b):
    d = (a - b).double()
    b = b.double()
    return float(max(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b), d.abs().max() / b.abs().max()))


def heat_pair(n, dirichlet, precision):
    mesh = W.Mesh(n, dirichlet=dirichlet)
    eps = 2.0 / max(n)
    dt = torch.float64 if precision == mf.MF_FP64 else torch.float32
    p = W.HeatParams(eps=eps)
    ctx = mf.Context(mesh)
    op = mf.heat_operator(ctx, p, phi=dev(W.phi_sphere(mesh, 0.3, eps), dt), precision=precision)
    return op, dev(W.uniform(0, mesh.n_nodes), dt)


def oseen_pair(n, dirichlet):
    mesh = W.Mesh(n, dirichlet=dirichlet)
    eps = 2.0 / max(n)
    p = W.OseenParams(eps=eps)
    ctx = mf.Context(mesh)
    op = mf.oseen_operator(ctx, p, dev(W.phi_wavy_plane(mesh, 0.5, 0.05, eps)), dev(W.taylor_green(mesh)))
    return op, dev(W.uniform(1, 3 * mesh.n_nodes))


CASES = [
    # (first call, second call on a smaller mesh, bar)
    ("heat fp64", lambda: heat_pair((64, 64, 64), W.ALL_FACES, mf.MF_FP64),
     lambda: heat_pair((9, 5, 7), W.FACE_XLO | W.FACE_ZHI, mf.MF_FP64), 1e-12),
    ("heat fp32", lambda: heat_pair((64, 64, 64), W.ALL_FACES, mf.MF_FP32),
     lambda: heat_pair((5, 6, 3), 0, mf.MF_FP32), 2e-6),
    ("oseen", lambda: oseen_pair((48, 48, 48), W.ALL_FACES), lambda: oseen_pair((6, 5, 9), W.FACE_YLO), 1e-12),
]


@pytest.mark.parametrize("name,first,second,tol", CASES, ids=[c[0] for c in CASES])
def test_noalloc_apply_matches_apply(gpu, name, first, second, tol):
    for make in (first, second):
        op, x = make()
        print(f"noalloc apply: {name}, {op.ctx.mesh.n} cells", flush=True)
        y_ref = torch.empty_like(x)
        mf.operator_apply(op, x, y_ref)
        y = torch.full_like(x, float("nan"))
        mf.operator_apply_noalloc(op, x, y)
        torch.cuda.synchronize()
        assert relerr(y, y_ref) <= tol
        assert torch.equal(y, y_ref)


def test_noalloc_apply_rejects_a_mesh_beyond_its_scratch(gpu):
    # 128^3 cells in FP64 need 32768 bricks * 891 slots * 8 bytes = 233 MB of
    # face-buffer scratch, more than the 64 MiB array: refused before any launch
    op, x = heat_pair((128, 128, 128), W.ALL_FACES, mf.MF_FP64)
    y = torch.zeros_like(x)
    with pytest.raises(mf.MFError, match="scratch"):
        mf.operator_apply_noalloc(op, x, y)
    assert float(y.abs().max()) == 0.0
    # the same mesh in FP32 at 96^3 (13824 bricks, 49 MB) fits
    op, x = heat_pair((96, 96, 96), W.ALL_FACES, mf.MF_FP32)
    y_ref = torch.empty_like(x)
    mf.operator_apply(op, x, y_ref)
    y = torch.empty_like(x)
    mf.operator_apply_noalloc(op, x, y)
    assert torch.equal(y, y_ref)
