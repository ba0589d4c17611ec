"""Pins for the oracle's flow diagnostics (kinetic energy, its rate, wall force).

  * E_K (Section 7.2 definition) is exact for a density that is constant and
    a momentum that is linear in x (the integrand is a polynomial the cubature
    integrates exactly) on any affine mesh, and reproduces the closed-form
    energy of the 2D and 3D Taylor-Green initial fields as h -> 0.
  * dE_K/dt (epsilon_1 = -dE_K/dt) equals the centred difference of E_K along
    the oracle's own SARK-4 trajectory on a moving mesh, to O(dt^2); it
    vanishes for a free stream on a moving mesh; the element Jacobian rate
    J div(w) equals the centred difference of J under the vertex motion.
  * Wall force (Section 7.3 c_D definition, Section 7.4 pressure / viscous
    split): a uniform pressure on a closed body gives zero force; a linear
    pressure gives the buoyancy -grad(p) |B| (divergence theorem, exact for the
    polynomial face quadrature); a uniform viscous stress gives zero; a linear
    one gives the volume integral of div(sigma).
"""
import math

import numpy as np
import pytest

from oracle import gbsystem as gb
from oracle.diagnostics import energy_rate, grid_divergence, kinetic_energy, wall_force
from oracle.mesh import Mesh
from oracle.motion import Motion
from oracle.rhs import Params, element_geometry
from oracle.solver import Solver
from workloads import kuhn_cube, make_case, ogrid_airfoil, periodic_square, taylor_green_2d, taylor_green_3d


def _moments_2d(rho, mx, my):
    return gb.equilibrium(2, rho, (mx / rho, my / rho), 1.0)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_kinetic_energy_exact_for_linear_momentum(N):
    """rho = 1.3, m = (a + b x + c y, d + e x + f y), c = 1 on the jittered
    periodic square [-1,1]^2: E_K = (1/(4 rho_inf)) * integral |m|^2 / (2 rho);
    the integral of (a + b x + c y)^2 over the square is 4a^2 + 4/3 (b^2 + c^2)."""
    vx, etov, per, _ = periodic_square(5, seed=2, jitter=0.15)
    mesh = Mesh(2, N, vx, etov, per)
    X = np.einsum("pv,kvd->kdp", mesh.ref.bary, vx[mesh.etov])
    a, b, c, d, e, f = 0.1, -0.2, 0.05, 0.03, 0.07, -0.11
    rho = np.full(X[:, 0].shape, 1.3)
    q = _moments_2d(rho, a + b * X[:, 0] + c * X[:, 1], d + e * X[:, 0] + f * X[:, 1]).transpose(1, 0, 2)
    EK, vol = kinetic_energy(mesh, Params(c=1.0, tau=1.0), q, vx, rho_inf=0.9)
    integral = (4 * a * a + 4 / 3 * (b * b + c * c) + 4 * d * d + 4 / 3 * (e * e + f * f)) / (2 * 1.3)
    assert abs(vol - 4.0) < 1e-14
    assert abs(EK - integral / (0.9 * 4.0)) < 1e-15


def test_kinetic_energy_of_taylor_green_2d():
    """u = u0 sin(pi x) cos(pi y), v = -u0 cos(pi x) sin(pi y), rho = 1 on
    [-1,1]^2: E_K = u0^2 / 4; the interpolated field converges to it."""
    u0 = 0.1
    errs = []
    for n in (4, 8):
        vx, etov, per, _ = periodic_square(n, seed=0, jitter=0.05)
        mesh = Mesh(2, 3, vx, etov, per)
        X = np.einsum("pv,kvd->kdp", mesh.ref.bary, vx[mesh.etov])
        rho, u = taylor_green_2d(X[:, 0], X[:, 1], u0)
        q = gb.equilibrium(2, rho, u, 1.0).transpose(1, 0, 2)
        EK, _ = kinetic_energy(mesh, Params(c=1.0, tau=1.0), q, vx)
        errs.append(abs(EK - u0 * u0 / 4) / (u0 * u0 / 4))
    assert errs[1] < 1e-3 and errs[1] < errs[0] / 6, errs


def test_kinetic_energy_of_taylor_green_3d():
    """Section 7.2 initial state on [-pi,pi]^3 with rho = 1: E_K = U0^2 / 8."""
    vx, etov, per, _ = kuhn_cube(4)
    mesh = Mesh(3, 3, vx, etov, per)
    X = np.einsum("pv,kvd->kdp", mesh.ref.bary, vx[mesh.etov])
    rho, u = taylor_green_3d(X[:, 0], X[:, 1], X[:, 2], 1.0)
    q = gb.equilibrium(3, rho, u, 1.0).transpose(1, 0, 2)
    EK, vol = kinetic_energy(mesh, Params(c=1.0, tau=1.0), q, vx)
    assert abs(vol - (2 * math.pi) ** 3) < 1e-10
    assert abs(EK - 0.125) < 2e-3


def test_jacobian_rate_is_j_times_divergence():
    """d/ds J(x + s w) at s = 0 equals J div(w) (J is quadratic in s for
    triangles, so the centred difference is exact)."""
    vx, etov, per, _ = periodic_square(4, seed=3, jitter=0.1)
    mesh = Mesh(2, 2, vx, etov, per)
    w = np.random.default_rng(5).normal(size=vx.shape)
    E = np.arange(mesh.K)
    J = element_geometry(mesh, vx, E)[0]
    h = 1e-3
    Jp = element_geometry(mesh, vx + h * w, E)[0]
    Jm = element_geometry(mesh, vx - h * w, E)[0]
    assert np.abs((Jp - Jm) / (2 * h) - J * grid_divergence(mesh, vx, w)).max() < 1e-12


def test_energy_rate_matches_difference_of_energy_along_trajectory():
    """-epsilon_1 = dE_K/dt at time t equals (E_K(t+dt) - E_K(t-dt)) / (2 dt)
    along the SARK-4 solution on the moving mesh, to O(dt^2): halving dt cuts
    the difference about four times."""
    cs = make_case("C1", n=6)
    mot = dict(cs.motion)
    kind = mot.pop("kind")
    diffs = []
    for dt in (4e-3, 2e-3):
        s = Solver(Mesh(2, 3, cs.vx, cs.etov, cs.period), Params(c=1.0, tau=0.02), Motion(kind, **mot))
        X = s.node_coords()
        rho, u = cs.macroscopic(X)
        s.set_state(gb.equilibrium(2, rho, u, 1.0).transpose(1, 0, 2))
        s.run(dt, int(round(0.1 / dt)) - 1)
        E0 = kinetic_energy(s.mesh, s.prm, s.q, s.x)[0]
        s.step(dt)
        rate = energy_rate(s.mesh, s.prm, s.q, s.x, s.motion.velocity(s.X, s.t))
        s.step(dt)
        E2 = kinetic_energy(s.mesh, s.prm, s.q, s.x)[0]
        diffs.append(abs((E2 - E0) / (2 * dt) - rate))
        assert abs(rate) > 1e-6
    assert diffs[1] < diffs[0] / 3.0 and diffs[1] < 1e-3 * abs(rate), (diffs, rate)


def test_energy_rate_of_free_stream_is_zero():
    """A uniform equilibrium state on the moving mesh: dE_K/dt = 0 (GCL)."""
    cs = make_case("C1_freestream", n=6)
    mot = dict(cs.motion)
    kind = mot.pop("kind")
    s = Solver(Mesh(2, 3, cs.vx, cs.etov, cs.period), Params(c=1.0, tau=0.01), Motion(kind, **mot))
    X = s.node_coords()
    rho, u = cs.macroscopic(X)
    q = gb.equilibrium(2, rho, u, 1.0).transpose(1, 0, 2)
    s.set_state(q)
    s.run(cs.dt, 5)
    EK, _ = kinetic_energy(s.mesh, s.prm, s.q, s.x)
    rate = energy_rate(s.mesh, s.prm, s.q, s.x, s.motion.velocity(s.X, s.t))
    assert abs(EK - 0.5 * (0.1 ** 2 + 0.1 ** 2)) < 1e-15
    assert abs(rate) < 1e-14


# ---------------------------------------------------------------- wall force

def _body_area(vx, etov, tag):
    """Area enclosed by the wall faces (shoelace over the wall edges, each
    oriented as in its fluid element, which runs clockwise around the body)."""
    area = 0.0
    for e, f in zip(*np.nonzero(tag == 1)):
        a, b = etov[e, f], etov[e, (f + 1) % 3]
        area += vx[a, 0] * vx[b, 1] - vx[b, 0] * vx[a, 1]
    return abs(0.5 * area)


@pytest.fixture(scope="module")
def airfoil():
    vx, etov, per, tag = ogrid_airfoil(4, 24)
    mesh = Mesh(2, 3, vx, etov, per, face_tag=tag)
    X = np.einsum("pv,kvd->kdp", mesh.ref.bary, vx[mesh.etov])
    return mesh, vx, X, _body_area(vx, etov, tag)


def test_uniform_pressure_gives_no_force(airfoil):
    mesh, vx, X, _ = airfoil
    rho = np.full(X[:, 0].shape, 1.2)
    q = _moments_2d(rho, 0 * rho, 0 * rho).transpose(1, 0, 2)
    Fp, Fv = wall_force(mesh, Params(c=0.7, tau=1.0), q, vx)
    assert np.abs(Fp).max() < 1e-15 and np.abs(Fv).max() == 0.0


def test_linear_pressure_gives_buoyancy(airfoil):
    """p = c^2 rho with rho = 1 + g.x: F_p = integral over the wall of p n,
    n pointing into the body, = -c^2 g |B|."""
    mesh, vx, X, area = airfoil
    g = np.array([0.3, -0.7])
    rho = 1.0 + g[0] * X[:, 0] + g[1] * X[:, 1]
    q = _moments_2d(rho, 0 * rho, 0 * rho).transpose(1, 0, 2)
    c = 0.7
    Fp, Fv = wall_force(mesh, Params(c=c, tau=1.0), q, vx)
    assert area > 0.05
    assert np.abs(Fp - (-c * c * g * area)).max() < 1e-14
    assert np.abs(Fv).max() == 0.0


def test_viscous_stress_force(airfoil):
    """sigma_xy = -c^2 (q4 - m_x m_y / rho) with m = 0: a uniform q4 gives no
    force; q4 = delta x gives F_v = integral over B of div(sigma) =
    (0, -c^2 delta |B|)."""
    mesh, vx, X, area = airfoil
    c, delta = 0.7, 0.01
    rho = np.ones(X[:, 0].shape)
    q = _moments_2d(rho, 0 * rho, 0 * rho)
    q[3] = delta
    Fp, Fv = wall_force(mesh, Params(c=c, tau=1.0), q.transpose(1, 0, 2), vx)
    assert np.abs(Fv).max() < 1e-16
    q[3] = delta * X[:, 0]
    Fp, Fv = wall_force(mesh, Params(c=c, tau=1.0), q.transpose(1, 0, 2), vx)
    assert np.abs(Fv - np.array([0.0, -c * c * delta * area])).max() < 1e-15
    # the normal stresses: S_xx = sqrt2 q5 = delta y gives (div sigma)_x = 0,
    # S_yy = sqrt2 q6 = delta y gives (div sigma)_y = -c^2 delta
    q[3] = 0.0
    q[5] = delta * X[:, 1] / math.sqrt(2)
    Fp, Fv = wall_force(mesh, Params(c=c, tau=1.0), q.transpose(1, 0, 2), vx)
    assert np.abs(Fv - np.array([0.0, -c * c * delta * area])).max() < 1e-15
