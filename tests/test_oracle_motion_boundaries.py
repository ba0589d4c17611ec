"""Pins for the oracle's mesh motions, boundary stand-ins and convergence.

  * Motions (Section 5; eq. gcl_exact_field, eq. TGV_deformation, the plunge
    of Section 7.3, the fish motion of Section 7.4): the grid velocity is the
    time derivative of the displacement (centred differences), the
    displacement takes the values the formulas fix at special points, and the
    RK4 vertex update reproduces X + d(X, t) at fourth order in dt.
  * Boundary stand-ins (wall ghost, far-field ghost, sponge): closed forms --
    a uniform state moving with a rigid wall gives F = 0 (zero relative normal
    mass flux, no jump), a uniform free stream gives F = 0 with far-field
    faces and the sponge, a uniform stress offset is damped by -sigma(r) delta.
  * Convergence of the moving-mesh solution at order >= N + 0.7 for
    N = 2, 3, 4 on 8^2, 16^2, 32^2 quads against the Fourier pseudo-spectral
    solution of the continuous system, with the mass integral kept to
    rounding on the moving mesh; in 3D, convergence of the moving tetrahedral
    solution to the spectral solution of the tensor-form system (written
    without the oracle's flux matrices) on the coarse meshes a CPU test
    affords.
"""
import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle import gbsystem as gb
from oracle.mesh import FARFIELD, WALL, Mesh
from oracle.motion import Motion, stage_positions
from oracle.rhs import Params, rhs
from oracle.solver import Solver
from workloads import kuhn_cube, ogrid_airfoil, periodic_square, taylor_green_2d
from workloads.fields import taylor_green_3d
from workloads.configs import cfl_dt

FISH = dict(a0=0.02, a1=-0.08, a2=0.16, lam=1.0, f=1.0, R_rigid=0.5, beta=10.0, T_ramp=1.0)

MOTIONS = [
    ("sin_product_2d", dict(A=(0.05, 0.03), T=1.0, L=(2.0, 2.0), origin=(0.1, -0.2)), 2),
    ("triple_product_3d", dict(A=0.03, T=20.0, L=2 * math.pi), 3),
    ("plunge_blend_2d", dict(h0=0.1, omega=0.7, r_in=1.5, r_out=16.0, center=(0.5, 0.0)), 2),
    ("fish_3d", FISH, 3),
]


def _points(dim, n=200, lo=-2.0, hi=2.0, seed=3):
    return np.random.default_rng(seed).uniform(lo, hi, size=(n, dim))


# ---------------------------------------------------------------- motions

@pytest.mark.parametrize("kind,p,dim", MOTIONS)
@pytest.mark.parametrize("t", [0.0, 0.23, 0.5, 1.7])
def test_velocity_is_time_derivative_of_displacement(kind, p, dim, t):
    m = Motion(kind, **p)
    X = _points(dim, lo=-3.0, hi=3.0) if kind != "plunge_blend_2d" else _points(dim, lo=-20, hi=20)
    h = 1e-5
    fd = (m.displacement(X, t + h) - m.displacement(X, t - h)) / (2 * h)
    v = m.velocity(X, t)
    scale = max(np.abs(v).max(), 1e-2)
    assert np.abs(fd - v).max() < 1e-8 * scale


def test_sin_product_special_values():
    """eq. gcl_exact_field with L = 2: at X = Y = 1/2 + origin and t = T/4 every
    sine is 1, so d = (Ax, Ay); on the lines X = origin + integer the
    displacement vanishes (periodic images stay matched)."""
    m = Motion("sin_product_2d", A=(0.05, 0.03), T=1.0, L=(2.0, 2.0), origin=(0.1, -0.2))
    d = m.displacement(np.array([[0.6, 0.3]]), 0.25)
    assert np.allclose(d, [[0.05, 0.03]], atol=1e-15)
    d = m.displacement(np.array([[0.1, 0.77], [1.1, -0.4], [-0.9, 0.5]]), 0.37)
    assert np.abs(d).max() < 1e-16


def test_triple_product_special_values():
    """eq. TGV_deformation on [-pi, pi]^3: d_x carries sin of the y and z
    phases only; at Y = Z = -pi/2 (phase -pi/2 + pi/2 ... = pi/2 after the
    shift by L/2) both are 1, so d_x = A sin(2 pi t / T)."""
    L, A, T = 2 * math.pi, 0.03, 20.0
    m = Motion("triple_product_3d", A=A, T=T, L=L)
    X = np.array([[0.7, -math.pi / 2, -math.pi / 2]])
    t = 3.0
    d = m.displacement(X, t)
    assert abs(d[0, 0] - A * math.sin(2 * math.pi * t / T)) < 1e-15
    # y- and z-components carry sin of the x phase: X + L/2 = 0.7 + pi
    sx = math.sin(2 * math.pi * (0.7 + L / 2) / L)
    assert abs(d[0, 1] - A * math.sin(2 * math.pi * t / T) * sx * 1.0) < 1e-15
    assert abs(d[0, 2] - A * math.sin(2 * math.pi * t / T) * sx * 1.0) < 1e-15


def test_plunge_special_values():
    """Section 7.3: y = Y - h0 sin(omega t), x = X inside the rigid zone; zero
    displacement beyond r_out; half the plunge at the middle of the ramp."""
    h0, om = 0.1, 0.7
    m = Motion("plunge_blend_2d", h0=h0, omega=om, r_in=1.5, r_out=16.0, center=(0.5, 0.0))
    t = 1.3
    X = np.array([[0.5, 0.0], [1.0, 0.3], [0.5 + 8.75, 0.0], [0.5, -17.0]])
    d = m.displacement(X, t)
    plunge = -h0 * math.sin(om * t)
    assert np.abs(d[:, 0]).max() == 0.0
    assert abs(d[0, 1] - plunge) < 1e-16 and abs(d[1, 1] - plunge) < 1e-16
    assert abs(d[2, 1] - 0.5 * plunge) < 1e-15
    assert d[3, 1] == 0.0


def test_fish_motion_printed_amplitudes():
    """Section 7.4: with a0 = 0.02, a1 = -0.08, a2 = 0.16 the peak-to-peak
    tail-beat amplitude is 0.2 body lengths (printed A_f / L = 0.2); the nose
    moves 0.04 peak to peak; only z moves; the ramp starts from rest and is
    complete at T_ramp; points within R_rigid of the body axis move with the
    axis (B = 1), points beyond it by exp(-beta d_eff^2)."""
    m = Motion("fish_3d", **FISH)
    ts = np.linspace(1.0, 2.0, 2001)                     # one period after the ramp
    X = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.3, 0.2, -0.3], [0.5, 0.9, 0.0]])
    D = np.stack([m.displacement(X, t) for t in ts])     # [t, point, dim]
    assert np.abs(D[:, :, :2]).max() == 0.0
    p2p = D[:, :, 2].max(axis=0) - D[:, :, 2].min(axis=0)
    assert abs(p2p[0] - 0.2) < 1e-6
    assert abs(p2p[1] - 0.04) < 1e-6
    # X = (1.3, 0.2, -0.3): clamped axis point 1, distance 0.5 = R_rigid -> B = 1
    assert abs(p2p[2] - 0.2) < 1e-6
    # X = (0.5, 0.9, 0): distance 0.9, d_eff = 0.4, B = exp(-1.6)
    A = 0.02 - 0.08 * 0.5 + 0.16 * 0.25
    assert abs(p2p[3] - 2 * A * math.exp(-10.0 * 0.16)) < 1e-6
    # ramp: at rest at t = 0, half-way at T_ramp / 2 (B = 1 at the tail)
    assert np.abs(m.displacement(X, 0.0)).max() == 0.0
    assert np.abs(m.velocity(X, 0.0)).max() == 0.0
    tail = np.array([[1.0, 0.0, 0.0]])
    t = 0.5
    assert abs(m.displacement(tail, t)[0, 2] - 0.5 * 0.1 * math.sin(2 * math.pi * (1.0 - t))) < 1e-15
    # continuity of displacement and velocity at the end of the ramp
    for f in (m.displacement, m.velocity):
        assert np.abs(f(X, 1.0 - 1e-9) - f(X, 1.0 + 1e-9)).max() < 1e-7


@pytest.mark.parametrize("kind,p,dim", MOTIONS)
def test_rk4_vertex_update_is_fourth_order(kind, p, dim):
    """Section 5: vertices advance by classical RK4 on dx/dt = v_G(X, t);
    after a fixed time they sit at X + d(X, t) up to O(dt^4)."""
    m = Motion(kind, **p)
    X = _points(dim, n=50, lo=-2.0, hi=2.0)
    Tend = 1.6 if kind != "triple_product_3d" else 12.0
    errs = []
    for nst in (8, 16, 32):
        dt = Tend / nst
        x = X.copy()
        for k in range(nst):
            _, _, x = stage_positions(m, X, x, k * dt, dt)
        errs.append(np.abs(x - (X + m.displacement(X, Tend))).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.7, (errs, rates)


# ---------------------------------------------------------------- boundary stand-ins

def _full_rate(s, q, F):
    """dq/dt = F - Lambda q (Section 4, eq. time_split)."""
    lam = gb.relaxation_rates(2, s.prm.tau)
    return F - lam[None, :, None] * q


def _airfoil_solver(N=2, motion=None, sponge=True, q_inf=None, n_r=6, n_theta=16):
    vx, etov, per, tag = ogrid_airfoil(n_r, n_theta)
    mesh = Mesh(2, N, vx, etov, per, face_tag=tag)
    sp = (0.5, 0.0, 10.0, 20.0, 2.0) if sponge else None
    return Solver(mesh, Params(c=1.0, tau=1e-3, q_inf=q_inf, sponge=sp), motion)


def test_wall_moving_with_uniform_state_gives_zero_rhs():
    """A uniform equilibrium state whose velocity equals the velocity of a
    rigidly plunging wall: the wall ghost equals the interior trace (zero
    relative normal mass flux, no-slip satisfied), so no face has a jump and
    F = 0 to rounding.  A ghost that ignored the wall velocity would not."""
    h0, om = 0.1, 0.7
    mot = Motion("plunge_blend_2d", h0=h0, omega=om, r_in=30.0, r_out=40.0, center=(0.5, 0.0))
    t = 0.9
    wy = -h0 * om * math.cos(om * t)
    q_inf = gb.equilibrium(2, np.array(1.0), (np.array(0.0), np.array(wy)), 1.0)
    s = _airfoil_solver(motion=mot, sponge=False, q_inf=q_inf)
    K, Np = s.mesh.K, s.mesh.ref.Np
    q = np.broadcast_to(q_inf[None, :, None], (K, 6, Np)).copy()
    w = mot.velocity(s.X, t)
    F = _full_rate(s, q, rhs(s.mesh, s.prm, q, s.x, w))
    assert np.abs(F).max() < 1e-12          # rounding of terms up to ~10 (fine wall layer, 1/tau)
    # the same state with a wall that does not move leaves a wall flux
    F0 = _full_rate(s, q, rhs(s.mesh, s.prm, q, s.x, np.zeros_like(w)))
    assert np.abs(F0).max() > 1e-3


def test_wall_ghost_mirrors_relative_normal_momentum():
    """At rest, a uniform state with momentum m: the wall flux of the density
    equation equals the upwinded jump in normal momentum, which vanishes only
    for tangential flow.  Checked through the mass integral: with a tangential
    free stream on a wall-bounded static mesh the density rate integrates to
    the far-field contribution only (here zero because q = q_inf)."""
    s = _airfoil_solver(sponge=False)
    K, Np = s.mesh.K, s.mesh.ref.Np
    q_inf = gb.equilibrium(2, np.array(1.0), (np.array(0.1), np.array(0.0)), 1.0)
    s.prm.q_inf = q_inf
    q = np.broadcast_to(q_inf[None, :, None], (K, 6, Np)).copy()
    F = rhs(s.mesh, s.prm, q, s.x, np.zeros_like(s.x))
    # mass rate = sum_e J 1^T M F_rho: no mass crosses a wall
    J = np.abs(np.linalg.det(np.stack([(s.x[s.mesh.etov][:, a + 1] - s.x[s.mesh.etov][:, 0]) / 2
                                       for a in range(2)], -1)))
    w1 = s.mesh.ref.M.sum(axis=0)
    mass_rate = np.einsum("k,p,kp->", J, w1, F[:, 0])
    assert abs(mass_rate) < 1e-13


def test_far_field_and_sponge_preserve_free_stream():
    """q = q_inf everywhere with far-field faces and the sponge: dq/dt = 0 to
    rounding on every element without a wall face (static and moving mesh;
    the free stream does not satisfy no-slip, so wall elements carry a flux)."""
    q_inf = gb.equilibrium(2, np.array(1.0), (np.array(0.1), np.array(0.02)), 1.0)
    for mot in (None, Motion("plunge_blend_2d", h0=0.1, omega=0.7, r_in=1.5, r_out=16.0, center=(0.5, 0.0))):
        s = _airfoil_solver(motion=mot, q_inf=q_inf)
        s.prm.flux_mode = "split"
        K, Np = s.mesh.K, s.mesh.ref.Np
        q = np.broadcast_to(q_inf[None, :, None], (K, 6, Np)).copy()
        w = s.motion.velocity(s.X, 0.4)
        F = _full_rate(s, q, rhs(s.mesh, s.prm, q, s.x, w))
        nowall = ~np.any(s.mesh.face_tag == WALL, axis=1)
        assert np.any(s.mesh.face_tag[nowall] == FARFIELD)
        assert np.abs(F[nowall]).max() < 1e-12


def test_sponge_damps_uniform_offset():
    """A uniform offset delta in the shear stress S_xy leaves the volume and
    interior-face terms at zero and Ntilde unchanged; on elements without a
    far-field face F_xy = -sigma(r) delta, with sigma = sigma_max ((r - r0) /
    (r1 - r0))^2 clipped to [0, sigma_max] at the node radius."""
    q_inf = gb.equilibrium(2, np.array(1.0), (np.array(0.1), np.array(0.0)), 1.0)
    s = _airfoil_solver(q_inf=q_inf, n_r=8, n_theta=16)
    K, Np = s.mesh.K, s.mesh.ref.Np
    delta = 3e-3
    q = np.broadcast_to(q_inf[None, :, None], (K, 6, Np)).copy()
    q[:, 3] += delta
    F = _full_rate(s, q, rhs(s.mesh, s.prm, q, s.x, np.zeros_like(s.x)))
    F[:, 3] += q[:, 3] / s.prm.tau - q_inf[3] / s.prm.tau    # keep the sponge part of F_xy only
    ff = np.any(s.mesh.face_tag != 0, axis=1)          # far-field and wall elements
    X = s.node_coords()
    r = np.hypot(X[:, 0] - 0.5, X[:, 1])
    sigma = 2.0 * np.clip((r - 10.0) / 10.0, 0.0, 1.0) ** 2
    expect = -sigma * delta
    assert np.any(sigma[~ff] > 0.5)
    assert np.abs(F[~ff, 3] - expect[~ff]).max() < 1e-13
    others = np.delete(F[~ff], 3, axis=1)
    assert np.abs(others).max() < 1e-13


# ---------------------------------------------------------------- convergence vs spectral

_CONV_T, _CONV_TAU, _CONV_U0 = 0.03, 0.05, 0.2


def _conv_errors(args):
    """(relative L2 error at t = T against the spectral solution, mass drift)
    of one (N, quads per side) run; executed in a worker process."""
    from tests.spectral_ref import Spectral2D
    N, n = args
    vx, etov, per, _ = periodic_square(n, seed=1, jitter=0.1)
    s = Solver(Mesh(2, N, vx, etov, per), Params(c=1.0, tau=_CONV_TAU),
               Motion("sin_product_2d", A=(0.05, 0.05), T=0.5, L=(2, 2)))
    X = s.node_coords()
    rho, u = taylor_green_2d(X[:, 0], X[:, 1], _CONV_U0)
    s.set_state(gb.equilibrium(2, rho, u, 1.0).transpose(1, 0, 2))
    m0 = s.integrals()
    nst = int(math.ceil(_CONV_T / cfl_dt(vx, etov, N, 1.0, 1.0, 0.25)))
    s.run(_CONV_T / nst, nst)
    sp = Spectral2D(48, 1.0, _CONV_TAU)
    Xs, Ys = np.meshgrid(sp.x, sp.x, indexing="xy")
    rho, u = taylor_green_2d(Xs, Ys, _CONV_U0)
    qT = sp.solve(gb.equilibrium(2, rho, u, 1.0), _CONV_T)
    X = s.node_coords()
    ref = sp.evaluate(qT, X[:, 0], X[:, 1]).transpose(1, 0, 2)
    err = s.l2_norm(s.q - ref)
    nrm = s.l2_norm(ref)
    rel = float(np.sqrt((err ** 2).sum()) / np.sqrt((nrm[1:3] ** 2).sum()))
    return rel, float(np.abs(s.integrals() - m0)[:3].max())


def test_moving_mesh_convergence_order_n_plus_one():
    """L2 error of the moving-mesh solution at t = 0.03 against the Fourier
    pseudo-spectral solution of the continuous system on 8^2, 16^2, 32^2
    split quads: observed order >= N + 0.7 for N = 2, 3, 4 on the finest pair.
    The mass integral sum_e J_e 1^T M rho_e stays at its initial value to
    rounding on the moving mesh (any truncation-level drift of the ALE form
    would also vanish under refinement)."""
    cases = [(N, n) for N in (2, 3, 4) for n in (8, 16, 32)]
    order = sorted(cases, key=lambda c: -(c[1] ** 2 * (c[0] + 1) ** 3))   # longest first
    workers = max(1, min(8, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = dict(zip(order, ex.map(_conv_errors, order)))
    for N in (2, 3, 4):
        errs = [res[(N, n)][0] for n in (8, 16, 32)]
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert rates[-1] >= N + 0.7, (N, errs, rates)
        assert min(rates) > N, (N, errs, rates)
        for n in (8, 16, 32):
            assert res[(N, n)][1] < 1e-13, (N, n, res[(N, n)][1])


_CONV3_T, _CONV3_TAU, _CONV3_U0 = 0.2, 0.05, 0.2


def _conv_errors_3d(args):
    """Relative L2 error at t = 0.2 of one (N, cubes per side) 3D run on
    [-pi, pi]^3 (Kuhn tetrahedra, triple-product motion) against the 3D
    spectral solution; executed in a worker process."""
    from tests.spectral_ref import Spectral3D
    N, n = args
    vx, etov, per, _ = kuhn_cube(n)
    s = Solver(Mesh(3, N, vx, etov, per), Params(c=1.0, tau=_CONV3_TAU),
               Motion("triple_product_3d", A=0.02, T=1.0, L=2 * math.pi))
    X = s.node_coords()
    rho, u = taylor_green_3d(X[:, 0], X[:, 1], X[:, 2], _CONV3_U0)
    s.set_state(gb.equilibrium(3, rho, u, 1.0).transpose(1, 0, 2))
    nst = int(math.ceil(_CONV3_T / cfl_dt(vx, etov, N, 1.0, 1.0, 0.25)))
    s.run(_CONV3_T / nst, nst)
    sp = Spectral3D(16, 1.0, _CONV3_TAU)
    Z, Y, Xs = np.meshgrid(sp.x, sp.x, sp.x, indexing="ij")
    rho, u = taylor_green_3d(Xs, Y, Z, _CONV3_U0)
    qT = sp.solve(gb.equilibrium(3, rho, u, 1.0), _CONV3_T)
    X = s.node_coords()
    ref = sp.evaluate(qT, X[:, 0], X[:, 1], X[:, 2]).transpose(1, 0, 2)
    err = s.l2_norm(s.q - ref)
    nrm = s.l2_norm(ref)
    return float(np.sqrt((err ** 2).sum()) / np.sqrt((nrm[1:4] ** 2).sum()))


def test_moving_mesh_convergence_3d():
    """The 3D moving-mesh solution converges to the continuous tensor-form
    system: N = 3 on 4^3 -> 8^3 cubes at order > 3.3 (observed 3.65), and,
    on coarser meshes, N = 1 (4^3 -> 8^3) and N = 2 (2^3 -> 4^3) at orders
    > 1.5 and > 2.0 (observed 1.62 and 2.22; k h = 1.6 and 0.8 per cube for
    the k = 1 vortex, pre-asymptotic).  The N = 3 pair resolves the model:
    dropping one flux-matrix entry (m_y through d_x S_xy) in a copy of the
    oracle leaves a 1.2 % error at 8^3 and an observed order of 0.85."""
    cases = [(3, 8), (1, 8), (3, 4), (1, 4), (2, 4), (2, 2)]       # longest first
    workers = max(1, min(6, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = dict(zip(cases, ex.map(_conv_errors_3d, cases)))
    for N, (a, b), floor in ((1, (4, 8), 1.5), (2, (2, 4), 2.0), (3, (4, 8), 3.3)):
        rate = math.log2(res[(N, a)] / res[(N, b)])
        assert rate > floor, (N, res, rate)
        assert res[(N, b)] < 0.25, (N, res)
