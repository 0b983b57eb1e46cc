"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only builds input data: node coordinates of the uniform Q2 grid,
level-set fields, convective fields, manufactured nodal fields and seeded
random vectors.  It holds none of the operator arithmetic (no basis functions,
no quadrature, no Heaviside, no property blending): both the GPU library and
the CPU oracle receive the arrays produced here and do that work themselves.

Node numbering of a mesh with ``n = (nx, ny, nz)`` cells is the Q2 node grid
``(2nx+1) x (2ny+1) x (2nz+1)`` with global id ``i + (2nx+1)*(j + (2ny+1)*k)``
(x fastest).  Vector fields are stored component-major (structure of arrays):
``[3][n_nodes]``.

Level-set profiles follow the initial condition of the paper's level-set
framework (Sec. 2.2, eq. initial_phi): phi = tanh(d / (2 eps)) with d a signed
distance that is positive in the liquid.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

# Face bits for homogeneous Dirichlet boundaries: bit f <-> face f.
FACE_XLO, FACE_XHI, FACE_YLO, FACE_YHI, FACE_ZLO, FACE_ZHI = (1 << i for i in range(6))
ALL_FACES = 0x3F


@dataclass(frozen=True)
class Mesh:
    """Uniform hexahedral mesh of a box split into ``n`` cells per direction."""

    n: Tuple[int, int, int]
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    dirichlet: int = 0  # bit mask of faces with homogeneous Dirichlet conditions

    @property
    def nodes_per_dim(self) -> Tuple[int, int, int]:
        return tuple(2 * c + 1 for c in self.n)

    @property
    def n_nodes(self) -> int:
        a, b, c = self.nodes_per_dim
        return a * b * c

    @property
    def n_cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))


def node_axes(mesh: Mesh):
    """1D node coordinates per direction (equispaced, spacing h/2)."""
    return [np.linspace(mesh.lo[d], mesh.hi[d], 2 * mesh.n[d] + 1) for d in range(3)]


def node_coords(mesh: Mesh) -> np.ndarray:
    """(n_nodes, 3) coordinates in global node order (x fastest)."""
    ax, ay, az = node_axes(mesh)
    Z, Y, X = np.meshgrid(az, ay, ax, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def uniform(seed: int, n: int) -> np.ndarray:
    """x ~ U[-1, 1] from numpy's default generator with the given seed."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def phi_sphere(mesh: Mesh, radius: float, eps: float, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """tanh profile of a liquid sphere: d = radius - |x - center| (liquid inside).

    Evaluated one z plane of nodes at a time (the same elementwise arithmetic
    as on the whole coordinate array), so that the largest meshes need no
    (n_nodes, 3) temporaries."""
    ax, ay, az = node_axes(mesh)
    Y, X = np.meshgrid(ay, ax, indexing="ij")
    pts = np.empty((X.size, 3))
    pts[:, 0], pts[:, 1] = X.ravel(), Y.ravel()
    c = np.asarray(center)[None, :]
    out = np.empty(mesh.n_nodes)
    for k, z in enumerate(az):
        pts[:, 2] = z
        d = radius - np.linalg.norm(pts - c, axis=1)
        out[k * X.size:(k + 1) * X.size] = np.tanh(d / (2.0 * eps))
    return out


def phi_wavy_plane(mesh: Mesh, z0: float, amp: float, eps: float) -> np.ndarray:
    """tanh profile of a liquid layer below z = z0 + amp cos(2 pi x) cos(2 pi y).

    d is the vertical distance to that surface (liquid below)."""
    x = node_coords(mesh)
    zs = z0 + amp * np.cos(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    return np.tanh((zs - x[:, 2]) / (2.0 * eps))


def taylor_green(mesh: Mesh) -> np.ndarray:
    """Divergence-free Taylor-Green vortex at the nodes, SoA [3][n_nodes].

    u = (sin(pi x) cos(pi y) cos(pi z), -cos(pi x) sin(pi y) cos(pi z), 0);
    its normal component vanishes on the faces of the unit cube."""
    x = node_coords(mesh)
    px, py, pz = np.pi * x[:, 0], np.pi * x[:, 1], np.pi * x[:, 2]
    u = np.empty((3, x.shape[0]))
    u[0] = np.sin(px) * np.cos(py) * np.cos(pz)
    u[1] = -np.cos(px) * np.sin(py) * np.cos(pz)
    u[2] = 0.0
    return u


def manufactured_T(mesh: Mesh) -> np.ndarray:
    """Nodal values of T = sin(pi x) sin(pi y) sin(pi z)."""
    x = node_coords(mesh)
    return np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2])


# ---------------------------------------------------------------------------
# Material data and workload presets
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class HeatParams:
    """Coefficients of the implicit heat operator rc/dt M + K(k).

    heaviside: 0 -> H = clamp((1 + phi)/2, 0, 1); 1 -> sine form in d(phi)."""

    k_l: float = 30.0
    k_g: float = 0.3
    rc_l: float = 5.0e6
    rc_g: float = 5.0e3
    dt: float = 1.0e-3
    heaviside: int = 0
    eps: float = 0.0  # interface thickness parameter (sine form only)

    @property
    def alpha_m(self) -> float:
        return 1.0 / self.dt

    alpha_k: float = 1.0
    alpha_c: float = 1.0  # factor of the convective term rho c_p u.grad T (used only with a velocity field)
    # three phases (used only with a nodal temperature for the coefficients):
    # solid conductivity and rho c_p, Ti-6Al-4V solidus and liquidus
    k_s: float = 20.0
    rc_s: float = 4.0e6
    T_sol: float = 1933.0
    T_liq: float = 2200.0
    penalty: float = 0.0  # Tanasawa penalty beta = alpha_v h_v (0: off)


@dataclass(frozen=True)
class OseenParams:
    """Coefficients of the linearized momentum operator rho/dt M + rho (u0.grad) + 2 mu eps:eps."""

    rho_l: float = 4000.0
    rho_g: float = 4.0
    mu_l: float = 5.0e-3
    mu_g: float = 5.0e-5
    dt: float = 1.0e-4
    heaviside: int = 0
    eps: float = 0.0
    alpha_c: float = 1.0
    alpha_v: float = 1.0
    # three phases (used only with a nodal temperature for the coefficients):
    # solid density and viscosity, melting range, Darcy damping C fs^2/((1-fs)^3+b)
    rho_s: float = 4200.0
    mu_s: float = 2.0e-2
    T_sol: float = 1933.0
    T_liq: float = 2200.0
    darcy_C: float = 1.0e8
    darcy_b: float = 1.0

    @property
    def alpha_m(self) -> float:
        return 1.0 / self.dt


def melt_temperature(mesh: Mesh) -> np.ndarray:
    """A frozen temperature field across the melting range of HeatParams:
    T = 1800 K + 600 K z (solid below z ~ 0.22, liquid above z ~ 0.67)."""
    return 1800.0 + 600.0 * node_coords(mesh)[:, 2]


@dataclass
class HeatWorkload:
    mesh: Mesh
    params: HeatParams
    phi: np.ndarray
    eps: float


def heat_sphere_workload(n: int, dirichlet: int, params: HeatParams | None = None) -> HeatWorkload:
    """Heat operator on the unit cube with a liquid sphere of radius 0.3 at the
    center, eps = 2h (h = cell edge)."""
    mesh = Mesh((n, n, n), dirichlet=dirichlet)
    eps = 2.0 / n
    p = params or HeatParams()
    return HeatWorkload(mesh, p, phi_sphere(mesh, 0.3, eps), eps)


@dataclass(frozen=True)
class SourceParams:
    """Interface heat sources: evaporative cooling (Tanasawa mass flux) and a
    Gaussian laser heat flux.  Material and laser values of the Ti-6Al-4V
    melt-pool setup (molar mass, boiling point, latent heat, vapor density;
    laser power and absorptivity); lengths are in units of the unit cube.

    terms: bit 0 evaporative cooling, bit 1 laser heat flux."""

    terms: int = 3
    evap_coeff: float = 1.0
    molar_mass: float = 4.78e-2
    vapor_density: float = 4.087
    T_boil: float = 3133.0
    h_v: float = 8.84e6
    power: float = 78.0
    absorptivity: float = 0.35
    radius: float = 0.1
    focus: tuple = (0.5, 0.5, 1.0)
    dir: tuple = (0.0, 0.0, -1.0)


@dataclass
class HeatSourceWorkload:
    mesh: Mesh
    params: HeatParams
    sources: SourceParams
    phi: np.ndarray
    T: np.ndarray
    eps: float


def heat_source_workload(n: int, dirichlet: int, params: HeatParams | None = None,
                         sources: SourceParams | None = None) -> HeatSourceWorkload:
    """Interface heat sources on the sphere level set of heat_sphere_workload,
    with a temperature field around the boiling point that peaks under the
    beam: T = T_v + 600 K exp(-((x-1/2)^2 + (y-1/2)^2) / 0.05) (z - 0.3)."""
    wl = heat_sphere_workload(n, dirichlet, params)
    sp = sources or SourceParams()
    x = node_coords(wl.mesh)
    T = sp.T_boil + 600.0 * np.exp(-((x[:, 0] - 0.5) ** 2 + (x[:, 1] - 0.5) ** 2) / 0.05) * (x[:, 2] - 0.3)
    return HeatSourceWorkload(wl.mesh, wl.params, sp, wl.phi, T, wl.eps)


@dataclass
class HeatConvWorkload:
    mesh: Mesh
    params: HeatParams
    phi: np.ndarray
    u0: np.ndarray
    eps: float


def heat_conv_workload(n: int, dirichlet: int, params: HeatParams | None = None,
                       speed: float = 1.0) -> HeatConvWorkload:
    """Heat operator with convection: the sphere level set of heat_sphere_workload
    and the Taylor-Green vortex (peak speed `speed`, m/s) as the velocity field."""
    wl = heat_sphere_workload(n, dirichlet, params)
    return HeatConvWorkload(wl.mesh, wl.params, wl.phi, speed * taylor_green(wl.mesh), wl.eps)


@dataclass
class OseenWorkload:
    mesh: Mesh
    params: OseenParams
    phi: np.ndarray
    u0: np.ndarray
    eps: float


def oseen_wavy_workload(n: int, dirichlet: int = ALL_FACES, params: OseenParams | None = None) -> OseenWorkload:
    """Oseen operator: liquid below z = 0.5 + 0.05 cos(2 pi x) cos(2 pi y),
    eps = 2h, Taylor-Green convective field, no-slip on all faces."""
    mesh = Mesh((n, n, n), dirichlet=dirichlet)
    eps = 2.0 / n
    return OseenWorkload(mesh, params or OseenParams(), phi_wavy_plane(mesh, 0.5, 0.05, eps),
                         taylor_green(mesh), eps)


@dataclass
class TransportWorkload:
    mesh: Mesh
    params: OseenParams
    sources: SourceParams
    phi: np.ndarray
    u: np.ndarray
    T: np.ndarray
    eps: float


def transport_workload(n: int, params: OseenParams | None = None,
                       sources: SourceParams | None = None) -> TransportWorkload:
    """Level-set transport velocity: the liquid sphere of radius 0.3 at the
    center (eps = 2h) with the sine Heaviside, the densities of OseenParams,
    the Taylor-Green velocity and a temperature around the boiling point of
    SourceParams, T = T_v + 300 K (z - 1/2) + 100 K cos(2 pi x) cos(2 pi y)."""
    mesh = Mesh((n, n, n))
    eps = 2.0 / n
    p = params or OseenParams(heaviside=1, eps=eps)
    sp = sources or SourceParams()
    x = node_coords(mesh)
    T = sp.T_boil + 300.0 * (x[:, 2] - 0.5) + 100.0 * np.cos(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    return TransportWorkload(mesh, p, sp, phi_sphere(mesh, 0.3, eps), taylor_green(mesh), T, eps)
