"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, exact integrals, invariants of the continuous operators,
textbook spectra, library routines and brute force on tiny meshes.

Each test names the mistake it is there to catch.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_2501_18781_amd import workloads as W

# Textbook 1D Q2 matrices on [0,1] (nodes 0, 1/2, 1).
M1 = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0
K1 = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3.0


def kron3(Az, Ay, Ax):
    """Matrix acting on local index a + 3b + 9c (x fastest)."""
    return np.kron(Az, np.kron(Ay, Ax))


class P:  # plain coefficient holder
    def __init__(self, **kw):
        self.__dict__.update(kw)


# ---------------------------------------------------------------------------
# Reference element
# ---------------------------------------------------------------------------

def test_gauss_rule_exact_to_degree_5_only():
    # catches: wrong points/weights, wrong interval mapping
    xi, w = O.gauss3()
    for p in range(6):
        assert abs(np.sum(w * xi ** p) - 1.0 / (p + 1)) < 1e-15
    assert abs(np.sum(w * xi ** 6) - 1.0 / 7) > 1e-5


def test_basis_1d_closed_forms():
    # l0 = 2x^2 - 3x + 1, l1 = -4x^2 + 4x, l2 = 2x^2 - x (expanded by hand)
    for x in [0.0, 0.5, 1.0, 0.1127, 0.37, 0.91]:
        v, d = O.basis1d(x)
        assert np.allclose(v, [2 * x * x - 3 * x + 1, -4 * x * x + 4 * x, 2 * x * x - x], atol=1e-15)
        assert np.allclose(d, [4 * x - 3, 4 - 8 * x, 4 * x - 1], atol=1e-14)


def test_cell_matrices_are_kronecker_products_of_1d_closed_forms():
    # catches: transposed/mis-ordered local numbering, wrong Jacobian scaling per direction
    h = (0.5, 2.0, 0.25)
    X = O.unit_cell_vertices(h)
    ones = np.ones(27)
    Mz, My, Mx = M1 * h[2], M1 * h[1], M1 * h[0]
    Kz, Ky, Kx = K1 / h[2], K1 / h[1], K1 / h[0]
    mass = O.heat_cell_matrix(X, None, kq27=ones, rcq27=ones, alpha_m=1.0, alpha_k=0.0)
    assert np.abs(mass - kron3(Mz, My, Mx)).max() < 1e-15
    stiff = O.heat_cell_matrix(X, None, kq27=ones, rcq27=ones, alpha_m=0.0, alpha_k=1.0)
    ref = kron3(Mz, My, Kx) + kron3(Mz, Ky, Mx) + kron3(Kz, My, Mx)
    assert np.abs(stiff - ref).max() < 1e-13 * np.abs(ref).max()


def test_affine_and_trilinear_cell_invariants():
    # catches: J^{-1} vs J^{-T} mix-ups, missing |det J|, sign errors in gradients
    rng = np.random.default_rng(7)
    B = np.array([[1.0, 0.3, -0.2], [0.1, 0.8, 0.25], [-0.15, 0.2, 1.2]])
    X = np.array([B @ np.array([(v >> d) & 1 for d in range(3)], float) for v in range(8)])
    Xt = X + 0.08 * rng.uniform(-1, 1, X.shape)  # non-affine trilinear cell
    for Xc, vol in [(X, abs(np.linalg.det(B))), (Xt, None)]:
        ones = np.ones(27)
        M = O.heat_cell_matrix(Xc, None, kq27=ones, rcq27=ones, alpha_m=1.0, alpha_k=0.0)
        K = O.heat_cell_matrix(Xc, None, kq27=ones, rcq27=ones, alpha_m=0.0, alpha_k=1.0)
        assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
        assert np.abs(K.sum(axis=1)).max() < 1e-13 * np.abs(K).max()   # constants have no gradient
        V = M.sum()
        if vol is not None:
            assert abs(V - vol) < 1e-14
        # u = a.x is trilinear in the reference coordinates, hence exact in Q2,
        # and its physical gradient is a at every quadrature point.
        nodes = np.array([[a / 2, b / 2, c / 2] for c in range(3) for b in range(3) for a in range(3)])
        phys = np.array([sum(Xc[v] * np.prod([(n[d] if (v >> d) & 1 else 1 - n[d]) for d in range(3)])
                             for v in range(8)) for n in nodes])
        a = np.array([0.7, -1.3, 0.4])
        u = phys @ a
        assert abs(u @ K @ u - (a @ a) * V) < 1e-12 * (a @ a) * V


# ---------------------------------------------------------------------------
# Pointwise coefficient functions (Sec. 2.3)
# ---------------------------------------------------------------------------

def test_heaviside_linear_form():
    H, dH = O.heaviside([-1.5, -1.0, -0.2, 0.0, 0.4, 1.0, 2.0], kind=0)
    assert np.allclose(H, [0, 0, 0.4, 0.5, 0.7, 1, 1], atol=1e-16)
    assert np.allclose(dH, [0, 0, 0.5, 0.5, 0.5, 0, 0])


def test_heaviside_sine_form_closed_values_and_derivative():
    eps = 0.05
    # d = 0 -> 1/2 ; d = +-3 eps -> 1, 0 ; d = 1.5 eps -> 3/4 + 1/(2 pi)
    phi_of_d = lambda d: np.tanh(d / (2 * eps))
    H, _ = O.heaviside([phi_of_d(0.0), phi_of_d(1.5 * eps), phi_of_d(-1.5 * eps),
                        phi_of_d(3.5 * eps), phi_of_d(-3.5 * eps)], kind=1, eps=eps)
    assert np.allclose(H, [0.5, 0.75 + 1 / (2 * np.pi), 0.25 - 1 / (2 * np.pi), 1.0, 0.0], atol=1e-13)
    # symmetry H(-phi) = 1 - H(phi) and dH by central differences
    phi = np.linspace(-0.89, 0.89, 41)
    Hp, dHp = O.heaviside(phi, 1, eps)
    Hm, _ = O.heaviside(-phi, 1, eps)
    assert np.allclose(Hp + Hm, 1.0, atol=1e-14)
    s = 1e-6
    fd = (O.heaviside(phi + s, 1, eps)[0] - O.heaviside(phi - s, 1, eps)[0]) / (2 * s)
    assert np.allclose(dHp, fd, rtol=1e-6, atol=1e-8)


def test_property_blends_with_constant_phi():
    # catches: swapped liquid/gas, arithmetic instead of reciprocal density (eqs. muEff, rhoEff)
    phi0 = 0.3
    Hc = 0.5 * (1 + phi0)
    p = W.HeatParams()
    X = O.unit_cell_vertices()
    A = O.heat_cell_matrix(X, p, phi27=np.full(27, phi0))
    k = Hc * p.k_l + (1 - Hc) * p.k_g
    rc = Hc * p.rc_l + (1 - Hc) * p.rc_g
    ref = p.alpha_m * rc * kron3(M1, M1, M1) + p.alpha_k * k * (
        kron3(M1, M1, K1) + kron3(M1, K1, M1) + kron3(K1, M1, M1))
    assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()
    q = W.OseenParams()
    Am = O.oseen_cell_matrix(X, q, np.full(27, phi0), np.zeros(81), alpha_c=0.0, alpha_v=0.0)
    rho = 1.0 / (Hc / q.rho_l + (1 - Hc) / q.rho_g)
    ref = q.alpha_m * rho * np.kron(np.eye(3), kron3(M1, M1, M1))
    assert np.abs(Am - ref).max() < 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Global heat operator
# ---------------------------------------------------------------------------

def _interp(mesh, f):
    x = W.node_coords(mesh)
    return f(x[:, 0], x[:, 1], x[:, 2])


def test_global_mass_sums_to_volume_and_stiffness_annihilates_constants():
    mesh = W.Mesh((3, 2, 4), lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 0.5))
    phi = W.uniform(3, mesh.n_nodes) * 0.9
    M = O.heat_matrix(mesh, W.HeatParams(), phi=phi, rc_l=1.0, rc_g=1.0, alpha_m=1.0, alpha_k=0.0)
    assert abs(M.sum() - 1.0) < 1e-13
    K = O.heat_matrix(mesh, W.HeatParams(), phi=phi, alpha_m=0.0, alpha_k=1.0)
    assert np.abs(K @ np.ones(mesh.n_nodes)).max() < 1e-12 * abs(K).max()
    assert abs(K - K.T).max() < 1e-13 * abs(K).max()


def test_quadratic_energy_closed_form():
    # u = x^2 y + z is exact in Q2: u^T A u = am rc int u^2 + ak k int |grad u|^2
    #   int u^2 = 1/15 + 1/6 + 1/3 = 17/30 ; int |grad u|^2 = 4/9 + 1/5 + 1 = 74/45
    mesh = W.Mesh((2, 3, 2))
    u = _interp(mesh, lambda x, y, z: x * x * y + z)
    ones = np.ones(mesh.n_cells * 27)
    A = O.heat_matrix(mesh, None, kq=2.5 * ones, rcq=0.75 * ones, alpha_m=3.0, alpha_k=1.0)
    ref = 3.0 * 0.75 * 17 / 30 + 2.5 * 74 / 45
    assert abs(u @ (A @ u) - ref) < 1e-13 * ref


def test_dirichlet_rows_are_identity_and_columns_removed():
    mesh = W.Mesh((2, 2, 2), dirichlet=W.FACE_XLO | W.FACE_ZHI)
    wl = W.heat_sphere_workload(2, 0)
    A = O.heat_matrix(mesh, wl.params, phi=wl.phi).toarray()
    cm = O.constrained_mask(mesh)
    x = W.node_coords(mesh)
    assert np.array_equal(cm, (x[:, 0] == 0.0) | (x[:, 2] == 1.0))
    assert np.array_equal(A[cm][:, cm], np.eye(cm.sum()))
    assert np.all(A[cm][:, ~cm] == 0) and np.all(A[~cm][:, cm] == 0)
    np.linalg.cholesky(A)  # SPD


def _l2_error(mesh, uh, ufun):
    """|| u_h - u ||_{L2} on a uniform unit-cube mesh, integrated cell by cell with
    numpy's 5-point Gauss-Legendre rule and the hand-expanded Q2 basis
    (independent of the oracle's own quadrature and basis code)."""
    n = mesh.n[0]
    h = 1.0 / n
    t, w = np.polynomial.legendre.leggauss(5)
    t, w = 0.5 * (t + 1), 0.5 * w
    B = np.stack([2 * t * t - 3 * t + 1, -4 * t * t + 4 * t, 2 * t * t - t], axis=1)  # [q, a]
    NX = 2 * n + 1
    U = uh.reshape(NX, NX, NX)
    # local 3x3x3 blocks of every cell: [cz, cy, cx, c, b, a]
    idx = 2 * np.arange(n)[:, None] + np.arange(3)[None, :]
    loc = U[idx[:, None, None, :, None, None], idx[None, :, None, None, :, None], idx[None, None, :, None, None, :]]
    uq = np.einsum("zc,yb,xa,ijkcba->ijkzyx", B, B, B, loc)
    c = np.arange(n) * h
    X = (c[None, None, :, None, None, None] + h * t[None, None, None, None, None, :])
    Y = (c[None, :, None, None, None, None] + h * t[None, None, None, None, :, None])
    Z = (c[:, None, None, None, None, None] + h * t[None, None, None, :, None, None])
    ww = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * h ** 3
    return np.sqrt(np.sum(ww[None, None, None] * (uq - ufun(X, Y, Z)) ** 2))


@pytest.mark.parametrize("variable", [False, True])
def test_manufactured_solution_converges_at_third_order(variable):
    # catches: dropped or sign-flipped terms, wrong coefficient evaluation
    # am rc T - div(k grad T) = f with T = sin(pi x) sin(pi y) sin(pi z), Dirichlet;
    # k and rc blended through H = (1 + phi)/2 of a tanh sphere profile (eps fixed).
    eps, R, c = 0.15, 0.3, np.array([0.513, 0.479, 0.507])  # center off the node grid
    p = P(k_l=3.0, k_g=1.0, rc_l=40.0, rc_g=20.0, alpha_m=1.0, alpha_k=1.0, heaviside=0, eps=0.0)
    Tfun = lambda x, y, z: np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)

    def fields(x):
        r = np.linalg.norm(x - c, axis=1)
        d = R - r
        phi = np.tanh(d / (2 * eps)) if variable else np.zeros(len(x))
        H = 0.5 * (1 + phi)
        k = p.k_g + (p.k_l - p.k_g) * H
        rc = p.rc_g + (p.rc_l - p.rc_g) * H
        gphi = ((1 - phi ** 2) / (2 * eps))[:, None] * (-(x - c) / r[:, None]) if variable else 0 * x
        gk = 0.5 * (p.k_l - p.k_g) * gphi
        s = np.sin(np.pi * x)
        co = np.cos(np.pi * x)
        T = s[:, 0] * s[:, 1] * s[:, 2]
        gT = np.pi * np.stack([co[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * co[:, 1] * s[:, 2],
                               s[:, 0] * s[:, 1] * co[:, 2]], axis=1)
        f = p.alpha_m * rc * T - (k * (-3 * np.pi ** 2 * T) + np.sum(gk * gT, axis=1))
        return phi, T, f

    errs = []
    for n in (4, 8, 16):
        mesh = W.Mesh((n, n, n), dirichlet=W.ALL_FACES)
        x = W.node_coords(mesh)
        phi, T, f = fields(x)
        A = O.heat_matrix(mesh, p, phi=phi)
        b = O.load_vector(mesh, fields(O.quad_points(mesh))[2])
        b[O.constrained_mask(mesh)] = 0.0
        Th = O.jacobi_cg(A, b, 1e-13).x
        errs.append(_l2_error(mesh, Th, Tfun))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.85), (errs, rates)


# ---------------------------------------------------------------------------
# Oseen operator
# ---------------------------------------------------------------------------

def test_oseen_viscous_term_kills_rigid_motions_and_matches_strain_energy():
    mesh = W.Mesh((2, 2, 3))
    nn = mesh.n_nodes
    phi = W.uniform(5, nn) * 0.9
    q = P(rho_l=1.0, rho_g=1.0, mu_l=2.0, mu_g=2.0, alpha_m=0.0, alpha_c=0.0, alpha_v=1.0)
    V = O.oseen_matrix(mesh, q, phi, np.zeros((3, nn)))
    x = W.node_coords(mesh)
    w = np.array([0.3, -0.7, 1.1])
    rigid = (np.array([1.0, 2.0, -0.5])[:, None] + np.cross(w, x).T).reshape(-1)
    assert np.abs(V @ rigid).max() < 1e-12 * abs(V).max()
    # u = (y^2, 0, x z): 2 mu int eps(u):eps(u) = 2 mu (2/3 + 1/6 + 1/3) = 7 mu / 3
    mesh1 = W.Mesh((2, 2, 2))
    x = W.node_coords(mesh1)
    u = np.stack([x[:, 1] ** 2, 0 * x[:, 0], x[:, 0] * x[:, 2]]).reshape(-1)
    V1 = O.oseen_matrix(mesh1, q, np.zeros(mesh1.n_nodes), np.zeros((3, mesh1.n_nodes)))
    assert abs(u @ (V1 @ u) - 7 * 2.0 / 3) < 1e-13


def test_oseen_convective_term_closed_forms():
    mesh = W.Mesh((2, 3, 2))
    nn = mesh.n_nodes
    x = W.node_coords(mesh)
    q = P(rho_l=1.0, rho_g=1.0, mu_l=0.0, mu_g=0.0, alpha_m=0.0, alpha_c=1.0, alpha_v=0.0)
    # u0 = (y, 0, 0), u = (x, 0, 0): int u . (u0 . grad) u = int x y = 1/4
    u0 = np.stack([x[:, 1], 0 * x[:, 0], 0 * x[:, 0]])
    C = O.oseen_matrix(mesh, q, np.zeros(nn), u0)
    u = np.concatenate([x[:, 0], np.zeros(nn), np.zeros(nn)])
    assert abs(u @ (C @ u) - 0.25) < 1e-14
    # constant u0 = a, u = (w.x) e_1: sum_i (C u)_i over component 1 = (a.w) |Omega|
    a, wv = np.array([0.4, -1.0, 2.0]), np.array([1.5, 0.5, -0.25])
    C2 = O.oseen_matrix(mesh, q, np.zeros(nn), np.repeat(a[:, None], nn, axis=1))
    u = np.concatenate([np.zeros(nn), x @ wv, np.zeros(nn)])
    y = C2 @ u
    assert abs(y[nn:2 * nn].sum() - a @ wv) < 1e-13
    assert np.abs(y[:nn]).max() == 0.0 and np.abs(y[2 * nn:]).max() == 0.0


def test_heat_convection_closed_forms_both_orientations():
    # The convective heat form c(f, g) = alpha_c int rc f (u0 . grad g) with the
    # linear field u0 = (y, 2z, 3x), f = x, g = x^2 + y^2 + z^2 (all exact in
    # Q2, integrands of degree <= 3 per direction, so the Gauss rule is exact):
    #   f^T C g = alpha_c rc int x (2xy + 4yz + 6xz) = alpha_c rc (1/3 + 1/2 + 1) = alpha_c rc 11/6
    #   g^T C f = alpha_c rc int (x^2 + y^2 + z^2) y                        = alpha_c rc 7/12
    # catches: N_i and grad N_j swapped (the two values trade places), wrong
    # sign, velocity components mixed up, u0 not interpolated at the points
    mesh = W.Mesh((2, 3, 2))
    x = W.node_coords(mesh)
    u0 = np.stack([x[:, 1], 2 * x[:, 2], 3 * x[:, 0]])
    ones = np.ones(mesh.n_cells * 27)
    rc, ac = 2.5, 1.5
    A = O.heat_matrix(mesh, None, kq=ones, rcq=rc * ones, u0=u0, alpha_m=0.0, alpha_k=0.0, alpha_c=ac)
    f = x[:, 0]
    g = (x ** 2).sum(axis=1)
    assert abs(f @ (A @ g) - ac * rc * 11 / 6) < 1e-13
    assert abs(g @ (A @ f) - ac * rc * 7 / 12) < 1e-13


def test_heat_convection_annihilates_constants_and_is_skew_with_dirichlet():
    # Sum_j N_j = 1, so C 1 = 0 for any velocity and coefficient (catches a
    # value instead of a derivative).  For constant u0 and rc, int v (u0 . grad w)
    # is skew for v, w vanishing on the boundary: with all faces Dirichlet the
    # symmetric part of A is exactly the operator without convection.
    wl = W.heat_conv_workload(3, 0)
    C = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi, u0=wl.u0, alpha_m=0.0, alpha_k=0.0)
    assert np.abs(C @ np.ones(wl.mesh.n_nodes)).max() < 1e-12 * abs(C).max()
    mesh = W.Mesh((3, 2, 3), dirichlet=W.ALL_FACES)
    nn = mesh.n_nodes
    phi = np.full(nn, 0.3)
    a = np.array([0.7, -1.3, 0.4])
    u0 = np.repeat(a[:, None], nn, axis=1)
    A = O.heat_matrix(mesh, W.HeatParams(), phi=phi, u0=u0, alpha_c=2.0e3)
    A0 = O.heat_matrix(mesh, W.HeatParams(), phi=phi)
    assert abs((A + A.T) / 2 - A0).max() < 1e-12 * abs(A0).max()
    assert abs(A - A.T).max() > 1e-3 * abs(A0).max()


# ---------------------------------------------------------------------------
# Interface heat sources (evaporative cooling, laser heat flux)
# ---------------------------------------------------------------------------

# gamma = 1, R/M = 1/(2 pi), rho_v = 1/2, T_v = 1, h_v = 1 make the Tanasawa
# coefficient 2/(2-1) * 1/sqrt(1) * (1/2)/1 = 1, so mdot = T - 1.
UNIT_EVAP = dict(evap_coeff=1.0, molar_mass=2 * np.pi * 8.314, vapor_density=0.5, T_boil=1.0, h_v=1.0)


def _linear_phi_case(n=(2, 3, 2), a=0.8, z0=0.5):
    # phi = a (z0 - z) stays inside (-1, 1): H = (1 + phi)/2, H' = 1/2, |grad phi| = a,
    # so delta = a/2 and rc = A + B z with A = rc_g + (rc_l - rc_g)(1 + a z0)/2,
    # B = -(rc_l - rc_g) a / 2; with rc_l = 3, rc_g = 1: c_rcp = 3/13.
    mesh = W.Mesh(n)
    x = W.node_coords(mesh)
    phi = a * (z0 - x[:, 2])
    p = W.HeatParams(rc_l=3.0, rc_g=1.0, heaviside=0)
    A, B = 1.0 + 2.0 * (1 + a * z0) / 2, -2.0 * a / 2
    return mesh, x, phi, p, a / 2, A, B, 3.0 / 13.0


def test_evaporative_cooling_closed_forms():
    # s = -mdot h_v delta rc c_rcp with mdot = tau: linear in z, so the Gauss
    # rule integrates the moments exactly:
    #   sum b = int s,  sum b z = int z s,  sum b x = int x s = (1/2) int s
    # catches: a wrong Tanasawa coefficient, delta without |grad phi|, the
    # blend of rc, z and x mixed up
    mesh, x, phi, p, delta, A, B, c = _linear_phi_case()
    tau = 2.0
    sp = W.SourceParams(terms=1, **UNIT_EVAP)
    b = O.heat_sources(mesh, p, sp, phi, np.full(mesh.n_nodes, 1.0 + tau))
    k = -tau * delta * c
    assert abs(b.sum() - k * (A + B / 2)) < 1e-13
    assert abs(b @ x[:, 2] - k * (A / 2 + B / 3)) < 1e-13
    assert abs(b @ x[:, 0] - k * (A + B / 2) / 2) < 1e-13
    # linear in T - T_v, zero at the boiling point
    b2 = O.heat_sources(mesh, p, sp, phi, np.full(mesh.n_nodes, 1.0 + 2 * tau))
    assert np.abs(b2 - 2 * b).max() < 1e-13 * np.abs(b).max()
    # (at T = T_v the interpolated T - T_v is a rounding residue)
    assert np.abs(O.heat_sources(mesh, p, sp, phi, np.ones(mesh.n_nodes))).max() < 1e-14 * np.abs(b).max()


def test_laser_flux_side_and_power():
    # flat liquid surface (phi > 0 below z0), normal n = -grad phi/|grad phi| = +e_z:
    # a beam pointing down (e_L = -e_z) is absorbed, one pointing up is not;
    # the absorbed power of a beam well inside the box is chi P (int delta_rcp dz)
    #   = chi P delta c (A + B/2) per unit area, with the Gaussian integrating to
    #   pi r^2 / 2 (tails beyond the box ~ exp(-50)); the centroid of b is the focus.
    mesh, x, phi, p, delta, A, B, c = _linear_phi_case(n=(2, 2, 2))
    up = W.SourceParams(terms=2, dir=(0.0, 0.0, 1.0))
    assert np.abs(O.heat_sources(mesh, p, up, phi, np.zeros(mesh.n_nodes))).max() == 0.0
    errs = []
    for n in (8, 16, 32):
        mesh, x, phi, p, delta, A, B, c = _linear_phi_case(n=(n, n, 2))
        sp = W.SourceParams(terms=2, radius=0.1, power=78.0, absorptivity=0.35, focus=(0.45, 0.55, 1.0))
        b = O.heat_sources(mesh, p, sp, phi, np.zeros(mesh.n_nodes))
        ref = 0.35 * 78.0 * delta * c * (A + B / 2)
        errs.append(abs(b.sum() - ref) / ref)
        cx, cy = (b @ x[:, 0]) / b.sum(), (b @ x[:, 1]) / b.sum()
    # Gauss rule on the Gaussian: fast convergence in h (3e-3, 9e-8, 5e-16 measured)
    assert errs[2] < 1e-10 and errs[1] < errs[0] / 100 and errs[2] < errs[1] / 100, errs
    assert abs(cx - 0.45) < 1e-10 and abs(cy - 0.55) < 1e-10


def test_sine_delta_integrates_to_one_across_a_flat_interface():
    # tanh profile, sine Heaviside: int delta f(H) dz = int_0^1 f(H) dH (co-area),
    # here f = -mdot h_v rc c_rcp with mdot = 2: sum b -> -2 c (rc_l + rc_g)/2 as h -> 0
    eps, errs = 0.04, []
    for n in (16, 32, 64):
        mesh = W.Mesh((1, 1, n))
        x = W.node_coords(mesh)
        phi = np.tanh((0.5 - x[:, 2]) / (2 * eps))
        p = W.HeatParams(rc_l=3.0, rc_g=1.0, heaviside=1, eps=eps)
        sp = W.SourceParams(terms=1, **UNIT_EVAP)
        b = O.heat_sources(mesh, p, sp, phi, np.full(mesh.n_nodes, 3.0))
        ref = -2.0 * (3.0 / 13.0) * (3.0 + 1.0) / 2
        errs.append(abs(b.sum() - ref) / abs(ref))
    # 3.7e-4, 6.1e-5, 1.2e-5 measured
    assert errs[2] < 5e-5 and errs[2] < errs[1] < errs[0], errs


def test_heat_sources_vanish_on_dirichlet_nodes():
    wl = W.heat_source_workload(3, W.FACE_ZHI | W.FACE_XLO)
    b = O.heat_sources(wl.mesh, wl.params, wl.sources, wl.phi, wl.T)
    cm = O.constrained_mask(wl.mesh)
    assert np.all(b[cm] == 0.0) and np.abs(b[~cm]).max() > 0.0


# ---------------------------------------------------------------------------
# Three phases (solid fraction from T), Darcy damping, Tanasawa penalty
# ---------------------------------------------------------------------------

def test_three_phase_coefficients_at_known_states():
    # With phi = 1 (dense) the heat matrix at a frozen temperature T equals the
    # matrix with the hand-computed constant coefficients (given per point):
    #   below the solidus: solid values; above the liquidus: liquid values;
    #   f_s = 1/2: H_s = 3/4 - 2/8 = 1/2; f_s = 1/4: H_s = 3/16 - 2/64 = 5/32;
    # with phi = -1 (gas) the gas values whatever T.
    # catches: f_s or H_s wrong (slope, ends), solid and liquid swapped
    mesh = W.Mesh((2, 2, 3))
    nn, nq = mesh.n_nodes, mesh.n_cells * 27
    p = W.HeatParams()
    ts, tl = p.T_sol, p.T_liq
    for T, phi0, Hs in [(ts - 50, 1.0, 1.0), (tl + 50, 1.0, 0.0), ((ts + tl) / 2, 1.0, 0.5),
                        (tl - (tl - ts) / 4, 1.0, 5 / 32), (ts - 50, -1.0, None)]:
        A = O.heat_matrix(mesh, p, phi=np.full(nn, phi0), Tc=np.full(nn, T))
        if Hs is None:
            k, rc = p.k_g, p.rc_g
        else:
            k, rc = Hs * p.k_s + (1 - Hs) * p.k_l, Hs * p.rc_s + (1 - Hs) * p.rc_l
        B = O.heat_matrix(mesh, p, kq=np.full(nq, k), rcq=np.full(nq, rc))
        assert abs(A - B).max() < 1e-13 * abs(B).max(), (T, phi0)


def test_darcy_damping_is_a_mass_term_of_the_solid():
    # Oseen with alpha_m = alpha_c = alpha_v = 0, phi = 1, at a frozen T: the
    # Darcy term is C fs^2 / ((1-fs)^3 + b) times the mass matrix per component:
    # fs = 1 -> C/b; fs = 1/2 -> C (1/4) / (1/8 + b); fs = 0 -> 0
    mesh = W.Mesh((2, 1, 2))
    nn = mesh.n_nodes
    q = W.OseenParams(darcy_C=3.0e5, darcy_b=0.5)
    M = O.heat_matrix(mesh, None, kq=np.ones(mesh.n_cells * 27), rcq=np.ones(mesh.n_cells * 27),
                      alpha_m=1.0, alpha_k=0.0).toarray()
    zero = np.zeros((3, nn))
    for T, K in [(q.T_sol - 10, 3.0e5 / 0.5), ((q.T_sol + q.T_liq) / 2, 3.0e5 * 0.25 / (0.125 + 0.5)),
                 (q.T_liq + 10, 0.0)]:
        D = O.oseen_matrix(mesh, q, np.ones(nn), zero, Tc=np.full(nn, T), alpha_m=0.0, alpha_c=0.0,
                           alpha_v=0.0).toarray()
        for c in range(3):
            blk = D[c * nn:(c + 1) * nn, c * nn:(c + 1) * nn]
            assert np.abs(blk - K * M).max() <= 1e-12 * max(K, 1.0) * np.abs(M).max()
        assert np.abs(D[:nn, nn:]).max() == 0.0


def test_oseen_three_phase_density_and_viscosity_reduce_to_two_phase():
    # At a uniform frozen temperature (H_s constant) and without Darcy damping
    # the three-phase Oseen matrix is the two-phase one with the liquid
    # values replaced by the solid-liquid blends rho_sl = H_s rho_s + (1 - H_s)
    # rho_l, mu_sl likewise (the two-phase path is pinned on its own); the
    # level set crosses the interface, so the reciprocal density blend and the
    # arithmetic viscosity blend are both exercised.
    # catches: rho blended arithmetically with gas, solid and liquid swapped,
    # H_s applied to the gas side
    mesh = W.Mesh((2, 3, 2), dirichlet=W.FACE_ZLO)
    nn = mesh.n_nodes
    q = W.OseenParams(darcy_C=0.0, mu_s=2.0e-2)  # solid values distinct from the liquid ones
    assert q.rho_s != q.rho_l and q.mu_s != q.mu_l
    phi = W.phi_wavy_plane(mesh, 0.5, 0.05, 0.25)
    u0 = W.taylor_green(mesh)
    for fs in (0.0, 0.3, 1.0):
        T = q.T_liq - fs * (q.T_liq - q.T_sol)
        Hs = 3 * fs ** 2 - 2 * fs ** 3
        A3 = O.oseen_matrix(mesh, q, phi, u0, Tc=np.full(nn, T))
        A2 = O.oseen_matrix(mesh, q, phi, u0, rho_l=Hs * q.rho_s + (1 - Hs) * q.rho_l,
                            mu_l=Hs * q.mu_s + (1 - Hs) * q.mu_l)
        assert abs(A3 - A2).max() <= 1e-13 * abs(A2).max(), fs


def test_penalty_term_moments_and_equivalence_with_evaporative_cooling():
    # Linear level set (delta = a/2, rc(z) = A + B z, see _linear_phi_case):
    # the penalty matrix R = beta delta_rcp N_i N_j has exact moments
    #   1^T R 1 = beta (a/2) c (A + B/2),  1^T R z = beta (a/2) c (A/2 + B/3);
    # and for any T, b_penalty(T_v) - R T equals the explicit evaporative
    # cooling with alpha_v h_v = beta (the penalty form of App. C).
    mesh, x, phi, p, delta, A, B, c = _linear_phi_case(n=(2, 2, 3))
    beta = 1.0  # = alpha_v h_v of UNIT_EVAP
    R = O.heat_matrix(mesh, p, phi=phi, alpha_m=0.0, alpha_k=0.0, penalty=beta)
    one = np.ones(mesh.n_nodes)
    assert abs(one @ (R @ one) - beta * delta * c * (A + B / 2)) < 1e-13
    assert abs(one @ (R @ x[:, 2]) - beta * delta * c * (A / 2 + B / 3)) < 1e-13
    T = 1.0 + W.uniform(5, mesh.n_nodes)
    b_pen = O.heat_sources(mesh, p, W.SourceParams(terms=4, **UNIT_EVAP), phi, T, penalty=beta)
    b_evap = O.heat_sources(mesh, p, W.SourceParams(terms=1, **UNIT_EVAP), phi, T)
    assert abs(b_pen.sum() - beta * 1.0 * delta * c * (A + B / 2)) < 1e-13
    assert np.abs(b_pen - R @ T - b_evap).max() < 1e-13 * np.abs(b_evap).max()


def test_spot_rows_agree_with_assembled_matrix():
    wl = W.heat_sphere_workload(3, W.FACE_YLO | W.FACE_ZHI)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    x = W.uniform(0, wl.mesh.n_nodes)
    rows = np.arange(0, wl.mesh.n_nodes, 5)
    y = A @ x
    assert np.abs(O.heat_rows(wl.mesh, wl.params, x, rows, phi=wl.phi) - y[rows]).max() < 1e-14 * np.abs(y).max()
    cw = W.heat_conv_workload(3, W.FACE_XHI | W.FACE_YLO)
    Ac = O.heat_matrix(cw.mesh, cw.params, phi=cw.phi, u0=cw.u0)
    for tr, ref in [(False, Ac @ x), (True, Ac.T @ x)]:
        got = O.heat_rows(cw.mesh, cw.params, x, rows, phi=cw.phi, u0=cw.u0, transpose=tr)
        assert np.abs(got - ref[rows]).max() < 1e-13 * np.abs(ref).max()
    ow = W.oseen_wavy_workload(2)
    B = O.oseen_matrix(ow.mesh, ow.params, ow.phi, ow.u0)
    x = W.uniform(1, B.shape[0])
    rows = np.arange(0, B.shape[0], 3)
    for tr, ref in [(False, B @ x), (True, B.T @ x)]:
        got = O.oseen_rows(ow.mesh, ow.params, ow.phi, ow.u0, x, rows, transpose=tr)
        assert np.abs(got - ref[rows]).max() < 1e-13 * np.abs(ref).max()


def test_csr_spmv_matches_sparse_product():
    # the oracle's own OpenMP CSR product (timed as the CPU baseline) against scipy's
    wl = W.heat_sphere_workload(5, W.ALL_FACES)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    x = W.uniform(4, wl.mesh.n_nodes)
    ref = A @ x
    assert np.abs(O.spmv(A, x) - ref).max() <= 1e-15 * np.abs(ref).max()


def test_block_jacobi_blocks_are_the_nodal_3x3_blocks():
    # read off the dense matrix by (component, node) index: block(i)[c][c'] = A[c nn + i, c' nn + i]
    ow = W.oseen_wavy_workload(2)
    nn = ow.mesh.n_nodes
    B = O.oseen_matrix(ow.mesh, ow.params, ow.phi, ow.u0)
    dense = B.toarray()
    bj = O.block_jacobi(B, nn)
    for i in (0, 7, nn // 2, nn - 1):
        blk = np.array([[dense[c * nn + i, cp * nn + i] for cp in range(3)] for c in range(3)])
        assert np.array_equal(bj.blocks[i], blk)
    assert np.allclose(np.einsum("nij,njk->nik", bj.inverse, bj.blocks), np.eye(3), atol=1e-12)
    # applying the preconditioner to B's own block-diagonal part returns the input
    v = W.uniform(5, 3 * nn)
    Dv = np.einsum("nij,nj->ni", bj.blocks, v.reshape(3, nn).T).T.reshape(-1)
    assert np.allclose(bj(Dv), v, atol=1e-12)


# ---------------------------------------------------------------------------
# Solvers
# ---------------------------------------------------------------------------

def test_cg_finite_termination_and_direct_agreement():
    # CG on a matrix with k distinct eigenvalues terminates in k steps
    d = np.repeat([1.0, 3.0, 7.0, 20.0], 25)
    import scipy.sparse as sps
    A = sps.diags(d).tocsr()
    b = W.uniform(11, d.size)
    r = O.jacobi_cg(A, b, 1e-12, dinv=np.ones(d.size))
    assert r.iters == 4 and np.allclose(r.x, b / d, rtol=1e-12)
    wl = W.heat_sphere_workload(4, W.ALL_FACES)
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    b = A @ W.uniform(0, wl.mesh.n_nodes)
    xs = O.direct_solve(A, b)
    r = O.jacobi_cg(A, b, 1e-14)
    assert r.converged and np.linalg.norm(r.x - xs) < 1e-12 * np.linalg.norm(xs)


def test_gmres_finite_termination_and_direct_agreement():
    import scipy.sparse as sps
    d = np.repeat([1.0, -2.0, 5.0], 20)
    A = (sps.diags(d) + sps.diags(0.0 * d[1:], 1)).tocsr()
    b = W.uniform(12, d.size)
    r = O.gmres(A, b, None, 30, 1e-12)
    assert r.iters == 3 and np.allclose(r.x, b / d)
    ow = W.oseen_wavy_workload(3)
    B = O.oseen_matrix(ow.mesh, ow.params, ow.phi, ow.u0)
    xs = W.uniform(1, B.shape[0])
    bj = O.block_jacobi(B, ow.mesh.n_nodes)
    r = O.gmres(B, B @ xs, bj, 30, 1e-13)
    ref = O.direct_solve(B, B @ xs)
    assert r.converged and np.linalg.norm(r.x - ref) < 1e-10 * np.linalg.norm(ref)
    # restart path: a tiny restart length still converges to the same solution
    r2 = O.gmres(B, B @ xs, bj, 5, 1e-12, maxit=2000)
    assert r2.converged and np.linalg.norm(r2.x - ref) < 1e-9 * np.linalg.norm(ref)


def test_chebyshev_matches_chebyshev_polynomial_closed_form():
    # error after m steps from zero: e_m(lam) = T_m((theta - lam)/delta) / T_m(theta/delta) e_0(lam)
    import scipy.sparse as sps
    from numpy.polynomial import chebyshev as C
    lam = np.linspace(0.2, 2.0, 40)
    A = sps.diags(lam).tocsr()
    xs = W.uniform(2, lam.size)
    b = lam * xs
    lmin, lmax = 0.1, 2.2
    th, de = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    for m in (1, 2, 4, 5):
        x = O.chebyshev_smooth(lambda v: A @ v, np.ones(lam.size), b, None, m, lmin, lmax)
        Tm = np.zeros(m + 1)
        Tm[m] = 1.0
        ref = C.chebval((th - lam) / de, Tm) / C.chebval(th / de, Tm) * xs
        assert np.allclose(xs - x, ref, atol=1e-13)


def test_lanczos_exact_on_full_krylov_space_and_laplacian_spectrum():
    import scipy.sparse as sps
    lam = np.array([0.5, 1.0, 2.0, 4.0, 4.5])
    A = sps.diags(lam).tocsr()
    est = O.lanczos_max_eig(lambda v: A @ v, np.ones(5), np.ones(5), steps=5)
    assert abs(est - 4.5) < 1e-12
    n = 60
    L = sps.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    est = O.lanczos_max_eig(lambda v: L @ v, np.full(n, 0.5), O.knuth_start_vector(n), steps=12)
    exact = 1 + np.cos(np.pi / (n + 1))
    assert est <= exact + 1e-12 and est > 0.97 * exact


def test_prolongation_reproduces_quadratics():
    mc = O.MeshDesc((2, 3, 2))
    mf = O.MeshDesc((4, 6, 4))
    P_ = O.prolongation(mc)
    f = lambda x, y, z: x * x * y - z * z + 0.5 * x * z + 1.0
    assert np.abs(P_ @ _interp(mc, f) - _interp(mf, f)).max() < 1e-14
    assert np.allclose(np.asarray(P_.sum(axis=1)).ravel(), 1.0)
    assert abs(O.inject(_interp(mf, f), mc) - _interp(mc, f)).max() == 0.0


def test_vcycle_is_symmetric_and_contracts():
    wl = W.heat_sphere_workload(8, W.ALL_FACES)
    levels = O.heat_mg_levels(wl.mesh, wl.params, wl.phi, n_coarse=2)
    assert [lv.mesh.n[0] for lv in levels] == [2, 4, 8]
    A = levels[-1].A
    a, b = W.uniform(21, A.shape[0]), W.uniform(22, A.shape[0])
    va, vb = O.vcycle(levels, a), O.vcycle(levels, b)
    assert abs(va @ b - a @ vb) < 1e-12 * abs(va @ b)
    # as a stationary iteration the V-cycle contracts the error strongly
    xs = W.uniform(23, A.shape[0])
    rhs = A @ xs
    x = O.vcycle(levels, rhs)
    x = x + O.vcycle(levels, rhs - A @ x)
    assert np.linalg.norm(x - xs) < 0.05 * np.linalg.norm(xs)
    r = O.flexible_cg(A, rhs, lambda v: O.vcycle(levels, v), rtol=1e-10)
    assert r.converged and r.iters <= 8 and np.linalg.norm(r.x - xs) < 1e-8 * np.linalg.norm(xs)


# ---------------------------------------------------------------------------
# Gradient of the one-step heat misfit
# ---------------------------------------------------------------------------

def _one_step(mesh, p, kq, rcq, Told):
    """T from A(k, rc) T = am M(rc) T_old (Dirichlet rows zero), by direct solve."""
    A = O.heat_matrix(mesh, p, kq=kq, rcq=rcq)
    Mrc = O.heat_matrix(mesh, p, kq=kq, rcq=rcq, alpha_k=0.0)
    b = Mrc @ Told
    b[O.constrained_mask(mesh)] = 0.0
    return A, O.direct_solve(A, b)


def test_gradient_formulas_match_brute_force_matrix_derivatives():
    # dL/dtheta = lam^T (db/dtheta - dA/dtheta T); A and b are linear in k_q and
    # rc_q, so unit perturbations give the exact derivative matrices.
    wl = W.heat_sphere_workload(2, W.ALL_FACES)
    mesh, p = wl.mesh, wl.params
    kq, rcq = O.heat_qp_coeffs(mesh, p, wl.phi)
    Told = W.manufactured_T(mesh)
    Told[O.constrained_mask(mesh)] = 0.0
    Ttgt = W.uniform(4, mesh.n_nodes) * 1e-3 + Told
    A, T = _one_step(mesh, p, kq, rcq, Told)
    cm = O.constrained_mask(mesh)
    g = 2 * (T - Ttgt)
    g[cm] = 0.0  # T is fixed on Dirichlet nodes: the adjoint sees only free residuals
    lam = O.direct_solve(A.T.tocsr(), g)
    dk, drc, _ = O.heat_grad(mesh, p, T, Told, lam)
    for q in [0, 13, 26, 27 * 3 + 5, 27 * 7 + 26]:
        e = np.zeros_like(kq)
        e[q] = 1.0
        dA = O.heat_matrix(mesh, p, kq=e, rcq=0 * e, alpha_m=0.0)
        dAk = dA.copy()
        g = -(lam @ (dAk @ T))
        assert abs(g - dk[q]) < 1e-10 * max(abs(g), np.abs(dk).max())
        dM = O.heat_matrix(mesh, p, kq=0 * e, rcq=e, alpha_k=0.0)
        # db - dA T with db = dM T_old on free rows; formed as dM (T_old - T)
        # because T - T_old is ~1e-7 of T in this mass-dominated step.
        db_dAT = dM @ (Told - T)
        db_dAT[cm] = 0.0
        g = lam @ db_dAT
        assert abs(g - drc[q]) < 1e-10 * max(abs(g), np.abs(drc).max())


def _one_step_delta(mesh, p, kq, rcq, Told):
    """Delta form of the step: A dT = -alpha_k K(k) T_old (zero on Dirichlet rows),
    T = T_old + dT.  Avoids the cancellation of forming T - T_old."""
    A = O.heat_matrix(mesh, p, kq=kq, rcq=rcq)
    K = O.heat_matrix(mesh, p, kq=kq, rcq=rcq, alpha_m=0.0)
    r = -(K @ Told)
    r[O.constrained_mask(mesh)] = 0.0
    return A, O.direct_solve(A, r)


def test_delta_form_equals_direct_step():
    wl = W.heat_sphere_workload(3, W.ALL_FACES)
    kq, rcq = O.heat_qp_coeffs(wl.mesh, wl.params, wl.phi)
    Told = W.manufactured_T(wl.mesh)
    Told[O.constrained_mask(wl.mesh)] = 0.0
    _, T = _one_step(wl.mesh, wl.params, kq, rcq, Told)
    _, dT = _one_step_delta(wl.mesh, wl.params, kq, rcq, Told)
    assert np.linalg.norm(T - (Told + dT)) < 1e-14 * np.linalg.norm(T)


def test_gradient_wrt_phi_matches_central_differences():
    wl = W.heat_sphere_workload(2, W.ALL_FACES)
    mesh, p = wl.mesh, wl.params
    cm = O.constrained_mask(mesh)
    Told = W.manufactured_T(mesh)
    Told[cm] = 0.0
    dTtgt = 1e-7 * W.uniform(4, mesh.n_nodes)
    dTtgt[cm] = 0.0

    def loss(phi):
        kq, rcq = O.heat_qp_coeffs(mesh, p, phi)
        _, dT = _one_step_delta(mesh, p, kq, rcq, Told)
        return np.sum((dT - dTtgt) ** 2), dT

    L0, dT = loss(wl.phi)
    kq, rcq = O.heat_qp_coeffs(mesh, p, wl.phi)
    A = O.heat_matrix(mesh, p, kq=kq, rcq=rcq)
    g = 2 * (dT - dTtgt)
    g[cm] = 0.0
    lam = O.direct_solve(A.T.tocsr(), g)
    _, _, dphi = O.heat_grad(mesh, p, Told + dT, Told, lam, phi=wl.phi)
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.uniform(-1, 1, mesh.n_nodes)
        s = 1e-6
        fd = (loss(wl.phi + s * v)[0] - loss(wl.phi - s * v)[0]) / (2 * s)
        assert abs(fd - dphi @ v) < 1e-6 * abs(fd)


# ---------------------------------------------------------------------------
# Whole steps with the Dirichlet nodes held at T_old
# ---------------------------------------------------------------------------

def test_heat_step_keeps_constants_steady_and_holds_boundary_values():
    # A constant temperature is a steady state of the step (K annihilates
    # constants), also where the Dirichlet nodes hold it.  Catches a missing
    # lifting of the boundary values: free rows that see 0 at the walls cool
    # the field next to them.
    wl = W.heat_sphere_workload(3, W.ALL_FACES)
    mesh, p = wl.mesh, wl.params
    kq, rcq = O.heat_qp_coeffs(mesh, p, wl.phi)
    n = mesh.n_nodes
    for delta in (True, False):
        T, _ = O.heat_step(mesh, p, np.full(n, 1234.5), kq=kq, rcq=rcq, delta=delta)
        assert np.abs(T - 1234.5).max() <= 1e-12 * 1234.5
    # A general field, nonzero on the walls: the delta and the plain form
    # agree, the Dirichlet nodes keep T_old, and the free rows satisfy
    # alpha_m M (T - T_old) + K T = 0 with every column present (a residual
    # of the assembled equation, not of either solve).
    cm = O.constrained_mask(mesh)
    Told = 2000.0 + 300.0 * W.manufactured_T(mesh) + 10.0 * W.uniform(5, n)
    T1, dT1 = O.heat_step(mesh, p, Told, kq=kq, rcq=rcq, delta=True)
    T2, _ = O.heat_step(mesh, p, Told, kq=kq, rcq=rcq, delta=False)
    assert np.linalg.norm(T1 - T2) <= 1e-14 * np.linalg.norm(T1)
    assert np.array_equal(T1[cm], Told[cm]) and not dT1[cm].any()
    m0 = O.without_dirichlet(mesh)
    M = O.heat_matrix(m0, p, kq=kq, rcq=rcq, alpha_k=0.0)
    K = O.heat_matrix(m0, p, kq=kq, rcq=rcq, alpha_m=0.0)
    res = (M @ dT1 + K @ T1)[~cm]
    assert np.abs(res).max() <= 1e-12 * np.abs(K @ T1).max()
    # with T_old = 0 on the walls it is the homogeneous step
    Told[cm] = 0.0
    _, T3 = _one_step(mesh, p, kq, rcq, Told)
    T4, _ = O.heat_step(mesh, p, Told, kq=kq, rcq=rcq, delta=False)
    assert np.linalg.norm(T3 - T4) <= 1e-14 * np.linalg.norm(T3)


def _three_phase_case(n=(4, 4, 4), dirichlet=W.ALL_FACES, penalty=2.0e9, dt=1e2):
    import dataclasses
    mesh = W.Mesh(n, dirichlet=dirichlet)
    eps = 2.0 / max(n)
    p = dataclasses.replace(W.HeatParams(eps=eps, penalty=penalty), dt=dt)
    phi = W.phi_sphere(mesh, 0.35, eps, center=(0.5, 0.5, 0.3))
    return mesh, p, phi, W.melt_temperature(mesh)


def test_picard_step_solves_the_nonlinear_step():
    # The converged iterate satisfies the nonlinear step itself,
    #   alpha_m M(T) (T - T_old) + (K + R)(T) T = b(T) on the free rows,
    # with the matrices evaluated at the final T (not at the iterate the last
    # solve used) and the Dirichlet nodes holding T_old.  Catches a lifting
    # that drops the boundary values, a right-hand side frozen at T_old, and
    # a penalty or source term missing from one side.
    import dataclasses
    mesh, p, phi, Told = _three_phase_case()
    sp = dataclasses.replace(W.SourceParams(), terms=7, radius=0.25)
    r = O.picard_step(mesh, p, phi, Told, sp, tol=1e-12, maxit=60)
    assert r.converged and r.iterations >= 3
    cm = O.constrained_mask(mesh)
    assert np.array_equal(r.T[cm], Told[cm])
    m0 = O.without_dirichlet(mesh)
    M = O.heat_matrix(m0, p, phi=phi, Tc=r.T, alpha_k=0.0, penalty=0.0)
    KR = O.heat_matrix(m0, p, phi=phi, Tc=r.T, alpha_m=0.0)
    b = O.heat_sources(mesh, p, sp, phi, r.T)
    res = (M @ (r.T - Told) + KR @ r.T - b)[~cm]
    assert np.abs(res).max() <= 1e-8 * np.abs(KR @ r.T).max()
    # T_old at the boiling temperature everywhere, penalty as the only term:
    # R T_v = b_penalty, so T_v is a steady state (first update exactly 0)
    Tv = np.full(mesh.n_nodes, sp.T_boil)
    r = O.picard_step(mesh, p, phi, Tv, dataclasses.replace(sp, terms=4), tol=1e-12, maxit=5)
    assert r.iterations == 1 and np.abs(r.T - sp.T_boil).max() <= 1e-9 * sp.T_boil


# ---------------------------------------------------------------------------
# Level-set transport velocity (Sec. 2.5, App. A)
# ---------------------------------------------------------------------------

def test_nodal_gradient_is_exact_for_q2_polynomials():
    # a field of degree <= 2 per direction is its own Q2 interpolant, so the
    # gradient at every node (every cell's one, and their average) is exact;
    # an off-diagonal product catches swapped directions and a wrong node order
    mesh = W.Mesh((3, 2, 4), lo=(-0.5, 0.0, 1.0), hi=(1.0, 0.5, 2.0))
    x, y, z = W.node_coords(mesh).T
    f = x * x * y - 3.0 * x * z + y * y * z * z + 2.0 * z
    g = O.nodal_gradient(mesh, f)
    ref = np.stack([2 * x * y - 3 * z, x * x + 2 * y * z * z, -3 * x + 2 * y * y * z + 2.0])
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_point_values_reproduce_q2_polynomials_and_clamp_to_the_box():
    mesh = W.Mesh((3, 2, 4), lo=(-0.5, 0.0, 1.0), hi=(1.0, 0.5, 2.0))
    x, y, z = W.node_coords(mesh).T
    fun = lambda x, y, z: x * x * y * z - 2.0 * y * z * z + x + 0.5
    pts = np.random.default_rng(3).uniform((-0.5, 0.0, 1.0), (1.0, 0.5, 2.0), (200, 3))
    pts = np.vstack([pts, [[-0.5, 0.0, 1.0], [1.0, 0.5, 2.0], [0.0, 0.25, 1.5]]])  # corners, cell faces
    v = O.point_values(mesh, fun(x, y, z), pts)
    assert np.abs(v - fun(*pts.T)).max() <= 1e-12
    # outside the box: the nearest point of the box
    out = np.array([[-1.0, 0.2, 1.5], [0.3, 0.9, 2.5], [2.0, -1.0, 0.0]])
    inside = np.clip(out, (-0.5, 0.0, 1.0), (1.0, 0.5, 2.0))
    assert np.abs(O.point_values(mesh, fun(x, y, z), out) - fun(*inside.T)).max() <= 1e-12


def _plane_case(a=(0.3, -0.2, -1.0), z0=0.55, eps=0.1, n=(4, 4, 6)):
    """Liquid below the oblique plane a.x = -z0 ... i.e. d = (z0 + a.x)/|a|
    (signed distance, liquid where d > 0), phi = tanh(d / 2 eps)."""
    mesh = W.Mesh(n)
    X = W.node_coords(mesh)
    a = np.asarray(a, float)
    d = (z0 + X @ a) / np.linalg.norm(a)
    p = W.OseenParams(heaviside=1, eps=eps)
    return mesh, X, d, np.tanh(d / (2 * eps)), p, a / np.linalg.norm(a)


def test_transport_projections_on_a_plane():
    # For a planar interface the recovered distance d(phi) is linear, its
    # nodal gradient exact, so n = grad d / |grad d| is the unit normal into
    # the liquid and the projections are closed forms: x_G = x - d n on the
    # plane, x_l = x + (3 eps - d) n on the parallel plane 3 eps into the
    # liquid.  Catches a flipped normal, a wrong projection distance and the
    # linear Heaviside's H = 1 contour.
    mesh, X, d, phi, p, nvec = _plane_case()
    sp = W.SourceParams()
    u = np.zeros((3, mesh.n_nodes))
    T = np.full(mesh.n_nodes, sp.T_boil)
    r = O.transport_velocity(mesh, p, sp, 2, phi, u, T)
    assert np.abs(r.normal - nvec[:, None]).max() <= 1e-12
    assert np.abs(r.x_gamma - (X - d[:, None] * nvec).T).max() <= 1e-12
    assert np.abs(r.x_liquid - (X + (3 * p.eps - d)[:, None] * nvec).T).max() <= 1e-12
    # on the plane and 3 eps into the liquid: d(x_G) = 0, d(x_l) = 3 eps
    dist = lambda P: (0.55 + P.T @ np.array([0.3, -0.2, -1.0])) / np.linalg.norm([0.3, -0.2, -1.0])
    assert np.abs(dist(r.x_gamma)).max() <= 1e-12
    assert np.abs(dist(r.x_liquid) - 3 * p.eps).max() <= 1e-12


def test_transport_projection_on_a_sphere_converges():
    # For a sphere the projected point x_G lands on the sphere up to the
    # second-order error of the nodal gradient of the interpolated distance;
    # on the band |d| < 3 eps with eps fixed: the error falls by about 4 when h halves
    errs = []
    for n in (8, 16, 32):
        mesh = W.Mesh((n, n, n))
        eps = 0.05
        phi = W.phi_sphere(mesh, 0.3, eps)
        X = W.node_coords(mesh)
        sp = W.SourceParams()
        r = O.transport_velocity(mesh, W.OseenParams(heaviside=1, eps=eps), sp, 2, phi,
                                 np.zeros((3, mesh.n_nodes)), np.full(mesh.n_nodes, sp.T_boil))
        band = np.abs(0.3 - np.linalg.norm(X - 0.5, axis=1)) < 3 * eps
        rad = np.linalg.norm(r.x_gamma.T[band] - 0.5, axis=1)
        errs.append(np.abs(rad - 0.3).max())
    assert errs[2] < 1e-3 and errs[1] / errs[2] > 3.0 and errs[0] / errs[1] > 3.0, errs


def test_transport_velocity_closed_forms_on_a_plane():
    mesh, X, d, phi, p, nvec = _plane_case()
    sp = W.SourceParams()
    gam = sp.evap_coeff
    alpha_v = 2 * gam / (2 - gam) * sp.h_v / np.sqrt(2 * np.pi * 8.314 / sp.molar_mass) * sp.vapor_density \
        / sp.T_boil ** 1.5
    # a velocity linear in x is reproduced exactly at x_l (variant 2); with
    # T = T_v there is no mass flux and variant 1 returns u itself
    A = np.array([[0.1, -0.3, 0.2], [0.05, 0.4, -0.1], [-0.2, 0.1, 0.3]])
    b = np.array([0.5, -1.0, 0.25])
    u = (X @ A.T + b).T
    Tv = np.full(mesh.n_nodes, sp.T_boil)
    r2 = O.transport_velocity(mesh, p, sp, 2, phi, u, Tv)
    xl = np.clip(r2.x_liquid.T, 0.0, 1.0)
    assert np.abs(r2.u_gamma - (xl @ A.T + b).T).max() <= 1e-12
    r1 = O.transport_velocity(mesh, p, sp, 1, phi, u, Tv)
    assert np.abs(r1.u_gamma - u).max() <= 1e-14
    # a temperature linear along the normal and quadratic along the plane:
    # variant 2's mass flux is its value at x_G, the same for every node of a
    # normal line (constant across the band), here alpha_v (T(x_G) - T_v)
    c1 = np.array([0.4, 0.7, 0.0])
    a = np.array([0.3, -0.2, -1.0])
    dist = lambda P: (0.55 + P @ a) / np.linalg.norm(a)
    Tfun = lambda P: sp.T_boil + 50.0 * (P @ c1) ** 2 + 80.0 * dist(P)
    r2 = O.transport_velocity(mesh, p, sp, 2, phi, np.zeros_like(u), Tfun(X))
    xg = np.clip(r2.x_gamma.T, 0.0, 1.0)  # projections that leave the box are moved back onto it
    inside = np.all(xg == r2.x_gamma.T, axis=1)
    assert inside.sum() > mesh.n_nodes // 2
    ref = alpha_v * (Tfun(xg) - sp.T_boil) / p.rho_l * nvec[:, None]
    assert np.abs(r2.u_gamma - ref).max() <= 1e-12 * np.abs(ref).max()
    # where x_G is inside the box, T(x_G) has no normal part: constant along normal lines
    assert np.abs(Tfun(xg[inside]) - sp.T_boil - 50.0 * (xg[inside] @ c1) ** 2).max() <= 1e-9
    T = Tfun(X)
    # variant 1 at H = 1 (deep in the liquid), H = 0 (gas) and H = 1/2 (on
    # the interface): mdot(T_j) / rho with the reciprocal blend's closed values
    r1 = O.transport_velocity(mesh, p, sp, 1, phi, np.zeros_like(u), T)
    mdot = alpha_v * (T - sp.T_boil)
    for sel, rho in [(d >= 3 * p.eps, p.rho_l), (d <= -3 * p.eps, p.rho_g)]:
        assert sel.any()
        ref = (mdot[sel] / rho) * nvec[:, None]
        assert np.abs(r1.u_gamma[:, sel] - ref).max() <= 1e-12 * np.abs(ref).max()
    mesh2, X2, d2, phi2, p2, nvec2 = _plane_case(a=(0.0, 0.0, -1.0), z0=0.5)
    on = np.abs(X2[:, 2] - 0.5) < 1e-12
    T2 = sp.T_boil + 100.0 * X2[:, 0]
    r1 = O.transport_velocity(mesh2, p2, sp, 1, phi2, np.zeros((3, mesh2.n_nodes)), T2)
    rho_half = 1.0 / (0.5 / p2.rho_l + 0.5 / p2.rho_g)
    ref = alpha_v * 100.0 * X2[on, 0] / rho_half
    assert np.abs(r1.u_gamma[2, on] + ref).max() <= 1e-12 * np.abs(ref).max()


def test_largest_stiffness_to_mass_diagonal_ratio():
    # the multigrid level rule bounds the stiffness part of the diagonal by
    # 17.5 (1/hx^2 + 1/hy^2 + 1/hz^2) times the mass part (unit coefficients):
    # a vertex node, (14/3) / (8/30) per direction; catches a wrong constant
    # (10, the midpoint ratio, or 30, the cell-centre node's)
    mesh = W.Mesh((3, 2, 4), lo=(0.0, 0.0, 0.0), hi=(1.0, 0.5, 2.0))
    unit = P(heaviside=0, k_l=1.0, k_g=1.0, rc_l=1.0, rc_g=1.0)
    phi = np.zeros(mesh.n_nodes)
    M = O.heat_matrix(mesh, unit, phi=phi, alpha_m=1.0, alpha_k=0.0).diagonal()
    K = O.heat_matrix(mesh, unit, phi=phi, alpha_m=0.0, alpha_k=1.0).diagonal()
    h = [(mesh.hi[d] - mesh.lo[d]) / mesh.n[d] for d in range(3)]
    bound = 17.5 * sum(1.0 / x ** 2 for x in h)
    assert abs((K / M).max() - bound) <= 1e-12 * bound
