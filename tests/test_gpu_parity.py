"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every input comes from the seeded generators in ``workloads`` (and the
oracle's equilibrium map); expected values come from the oracle only.
Tolerances: FP64 1e-12 relative per field, both in the L2 norm and element
by element against the field's largest entry; FP32 (perturbation storage
q1 - rho0) 1e-5 relative on the velocity, looser bounds stated per test for
raw right-hand sides.
"""
import math

import numpy as np
import pytest

from oracle import gbsystem as gb
from oracle.mesh import Mesh
from oracle.motion import Motion
from oracle.rhs import Params, rhs as oracle_rhs
from oracle.solver import Solver
from workloads import make_case, kuhn_cube, ogrid_airfoil
from workloads.configs import cfl_dt

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2607_00199_amd")
from paper_2607_00199_amd import _lib as L  # noqa: E402
from paper_2607_00199_amd.session import Session  # noqa: E402


def _oracle_for(case, mode="split", **kw):
    mesh = Mesh(case.dim, case.N, case.vx, case.etov, case.period, face_tag=case.face_tag)
    mot = dict(case.motion)
    kind = mot.pop("kind")
    return Solver(mesh, Params(c=case.c, tau=case.tau, flux_mode=mode, **kw), Motion(kind, **mot))


def _state(osolver, case, perturb=0.0, seed=0):
    X = osolver.node_coords()
    rho, u = case.macroscopic(X)
    q = gb.equilibrium(case.dim, rho, u, case.c).transpose(1, 0, 2).copy()
    if case.init == "decay":
        q[:, case.dim + 1:] += case.extra["delta"]
    if perturb:
        rng = np.random.default_rng(seed)
        q += perturb * rng.standard_normal(q.shape) * np.abs(q).max(axis=(0, 2))[None, :, None]
    return q


def _rel(a, b):
    """Largest per-field relative difference, taking the larger of two
    measures for each field: the L2 norm of the difference over the L2 norm
    of the reference, and the element-wise maximum of |a - b| over the
    largest |b| of that field (a field that is zero in the reference is
    measured against the largest entry of any field)."""
    out = 0.0
    top = np.abs(b).max()
    for f in range(a.shape[1]):
        nrm = np.linalg.norm(b[:, f])
        if nrm > 0:
            out = max(out, np.linalg.norm(a[:, f] - b[:, f]) / nrm)
        scale = np.abs(b[:, f]).max()
        out = max(out, np.abs(a[:, f] - b[:, f]).max() / (scale if scale > 0 else top))
    return out


def test_library_is_native():
    assert L.load() is not None
    assert "gfx950" in L.gb_version()


@pytest.mark.parametrize("name,kw", [("C1", {}), ("C2_small", {}), ("C3", {"n": 3})])
def test_nodes_match_oracle(name, kw):
    case = make_case(name, **kw)
    s = Session(case)
    o = _oracle_for(case)
    assert np.abs(s.nodes() - o.node_coords()).max() < 1e-12
    s.close()


@pytest.mark.parametrize("mode,flux", [("split", L.GB_FLUX_SPLIT), ("relative", L.GB_FLUX_RELATIVE)])
def test_rhs_parity_fp64_2d(mode, flux):
    case = make_case("C1", n=8)
    s = Session(case, flux_mode=flux)
    o = _oracle_for(case, mode)
    q = _state(o, case, perturb=1e-3)
    Fg = s.rhs(q)
    Fo = o.rhs_now(q)
    assert _rel(Fg, Fo) < 1e-12
    s.close()


def test_rhs_parity_fp64_2d_moving_time():
    """Right-hand side at t > 0 (nonzero grid velocity) after the state was
    set with that time: exercises the ALE terms."""
    case = make_case("C1", n=8)
    s = Session(case)
    o = _oracle_for(case)
    q = _state(o, case, perturb=1e-3, seed=3)
    t0 = 0.13
    s.set_state(q, t0)
    o.set_state(q, t0)
    Fg = s.rhs(q)
    Fo = o.rhs_now(q)
    assert _rel(Fg, Fo) < 1e-12
    s.close()


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_rhs_parity_fp64_orders(N):
    case = make_case("C2_small", n=6, N=N)
    s = Session(case)
    o = _oracle_for(case)
    q = _state(o, case, perturb=1e-3, seed=N)
    assert _rel(s.rhs(q), o.rhs_now(q)) < 1e-12
    s.close()


def test_rhs_parity_fp32_2d():
    case = make_case("C2_small", n=8)
    s = Session(case, precision=L.GB_FP32)
    o = _oracle_for(case)
    q = _state(o, case, perturb=1e-4, seed=5)
    Fg, Fo = s.rhs(q), o.rhs_now(q)
    # FP32 arithmetic on O(1e-1) momenta and O(1e-3) stresses: relative to the
    # largest entry of each field
    for f in range(6):
        assert np.abs(Fg[:, f] - Fo[:, f]).max() < 2e-5 * np.abs(Fo[:, f]).max(), f
    s.close()


@pytest.mark.parametrize("mode,flux", [("split", L.GB_FLUX_SPLIT), ("relative", L.GB_FLUX_RELATIVE)])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_rhs_parity_fp64_3d(N, mode, flux):
    case = make_case("C3", n=3, N=N)
    s = Session(case, flux_mode=flux)
    o = _oracle_for(case, mode)
    q = _state(o, case, perturb=1e-3, seed=N)
    s.set_state(q, 2.0)
    o.set_state(q, 2.0)
    assert _rel(s.rhs(q), o.rhs_now(q)) < 1e-12
    s.close()


@pytest.mark.parametrize("dim,N", [(2, 1), (3, 1), (3, 3)])
def test_rhs_parity_fp32_thin_last_tile(dim, N):
    """FP32 shapes whose last 16-row node tile holds at most four real rows
    (contracted by 4x4x1 blocks with the contraction split across lanes):
    right-hand side within 2e-5 of each field's largest entry, both flux
    modes, on a moving mesh at t = 0.7."""
    for mode, flux in (("split", L.GB_FLUX_SPLIT), ("relative", L.GB_FLUX_RELATIVE)):
        case = make_case("C2_small", n=6, N=N) if dim == 2 else make_case("C3", n=3, N=N)
        s = Session(case, precision=L.GB_FP32, flux_mode=flux)
        o = _oracle_for(case, mode)
        q = _state(o, case, perturb=1e-4, seed=13)
        s.set_state(q, 0.7)
        o.set_state(q, 0.7)
        Fg, Fo = s.rhs(q), o.rhs_now(q)
        for f in range(Fo.shape[1]):
            assert np.abs(Fg[:, f] - Fo[:, f]).max() < 2e-5 * np.abs(Fo).max(), (mode, f)
        s.close()


@pytest.mark.parametrize("dim,mode,flux", [(2, "relative", L.GB_FLUX_RELATIVE), (3, "split", L.GB_FLUX_SPLIT),
                                           (3, "relative", L.GB_FLUX_RELATIVE)])
def test_rhs_parity_fp32_modes(dim, mode, flux):
    """FP32 right-hand side in both flux modes, 2D and 3D (N = 3), within
    2e-5 of each field's largest entry."""
    case = make_case("C2_small", n=6, N=3) if dim == 2 else make_case("C3", n=3, N=3)
    s = Session(case, precision=L.GB_FP32, flux_mode=flux)
    o = _oracle_for(case, mode)
    q = _state(o, case, perturb=1e-4, seed=11)
    s.set_state(q, 0.7)
    o.set_state(q, 0.7)
    Fg, Fo = s.rhs(q), o.rhs_now(q)
    for f in range(Fo.shape[1]):
        assert np.abs(Fg[:, f] - Fo[:, f]).max() < 2e-5 * np.abs(Fo).max(), f
    s.close()


def test_rhs_parity_boundaries_and_sponge():
    """O-grid with wall and far-field faces and the sponge layer (stand-ins,
    parity against the oracle's stand-ins only)."""
    vx, etov, per, tag = ogrid_airfoil(6, 24, radius=6.0)
    case = make_case("C4")
    case.vx, case.etov, case.period, case.face_tag = vx, etov, per, tag
    case.motion = dict(case.motion, r_in=1.0, r_out=4.0)
    q_inf = gb.equilibrium(2, np.array(1.0), [np.array(0.1), np.array(0.0)], 1.0)
    sponge = (0.5, 0.0, 4.5, 6.0, 2.0)
    s = Session(case, q_inf=q_inf, sponge=sponge)
    o = _oracle_for(case, q_inf=q_inf, sponge=sponge)
    q = _state(o, case, perturb=1e-3, seed=9)
    s.set_state(q, 0.3)
    o.set_state(q, 0.3)
    assert _rel(s.rhs(q), o.rhs_now(q)) < 1e-12
    s.close()


# vertices of face f of a tetrahedron (the face opposite the fourth entry)
_TET_FACES = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def _walled_box_3d(N):
    """Non-periodic tetrahedral box [-0.6, 1.4]^3 on the moving 3D workload:
    boundary faces below z = 0.4 are walls, the rest far field."""
    vx, etov, _, _ = kuhn_cube(3, lo=-0.6, hi=1.4)
    tag = np.zeros((etov.shape[0], 4), np.int8)
    for f, vs in enumerate(_TET_FACES):
        zc = vx[etov[:, list(vs)], 2].mean(axis=1)
        tag[:, f] = np.where(zc < 0.4, L.GB_FACE_WALL, L.GB_FACE_FARFIELD)
    case = make_case("C3", n=3, N=N)
    case.vx, case.etov, case.period, case.face_tag = vx, etov, None, tag
    q_inf = gb.equilibrium(3, np.array(1.0), [np.array(0.1), np.array(0.0), np.array(0.0)], case.c)
    return case, q_inf


@pytest.mark.parametrize("N", [1, 2, 3])
def test_rhs_parity_boundaries_3d(N):
    """Tetrahedra with wall and far-field faces on a moving mesh (every
    element has boundary faces on some of its lane quarters' faces): FP64
    right-hand side within 1e-12 of the oracle's, both flux modes; FP32 at
    the order of the 3D workload within 2e-5 of each field's largest entry."""
    case, q_inf = _walled_box_3d(N)
    for mode, flux in (("split", L.GB_FLUX_SPLIT), ("relative", L.GB_FLUX_RELATIVE)):
        o = _oracle_for(case, mode, q_inf=q_inf)
        q = _state(o, case, perturb=1e-3, seed=20 + N)
        o.set_state(q, 1.3)
        Fo = o.rhs_now(q)
        s = Session(case, flux_mode=flux, q_inf=q_inf)
        s.set_state(q, 1.3)
        assert _rel(s.rhs(q), Fo) < 1e-12, mode
        s.close()
        if N == 3:
            s = Session(case, precision=L.GB_FP32, flux_mode=flux, q_inf=q_inf)
            s.set_state(q, 1.3)
            Fg = s.rhs(q)
            for f in range(Fo.shape[1]):
                assert np.abs(Fg[:, f] - Fo[:, f]).max() < 2e-5 * np.abs(Fo[:, f]).max(), (mode, f)
            s.close()


def _run_both(case, nsteps, precision=L.GB_FP64, mode="split", graph=False):
    flux = L.GB_FLUX_SPLIT if mode == "split" else L.GB_FLUX_RELATIVE
    s = Session(case, precision=precision, flux_mode=flux)
    o = _oracle_for(case, mode)
    q0 = _state(o, case)
    s.set_state(q0)
    o.set_state(q0)
    s.step(case.dt, nsteps, graph=graph)
    qg, t, step = s.get_state()
    o.run(case.dt, nsteps)
    xg = L.gb_mesh_vertices(s.mesh, case.vx.shape[0], case.dim)
    s.close()
    return qg, o, t, step, xg


def test_sark_c1_full_fp64():
    """The 2D moving Taylor-Green configuration: 512 triangles, N=3, 200 SARK
    steps; GPU FP64 within 1e-12 of the oracle."""
    case = make_case("C1")
    qg, o, t, step, xg = _run_both(case, case.nsteps)
    assert step == case.nsteps and abs(t - o.t) < 1e-14
    assert np.abs(xg - o.x).max() < 1e-14
    assert _rel(qg, o.q) < 1e-12


def test_sark_relative_flux_fp64():
    case = make_case("C1", n=8)
    qg, o, *_ = _run_both(case, 40, mode="relative")
    assert _rel(qg, o.q) < 1e-12


def test_graph_replay_matches_eager():
    case = make_case("C1", n=8)
    a = Session(case)
    b = Session(case)
    q0 = a.initial_state()
    a.set_state(q0)
    b.set_state(q0)
    for _ in range(3):
        a.step(case.dt, 5)
        b.step(case.dt, 5, graph=True)
        qa, ta, _ = a.get_state()
        qb, tb, _ = b.get_state()
        assert np.array_equal(qa, qb) and ta == tb
    a.close()
    b.close()


def test_free_stream_gpu():
    case = make_case("C1_freestream")
    s = Session(case)
    q0 = s.initial_state()
    s.set_state(q0)
    s.step(case.dt, 100)
    q, *_ = s.get_state()
    assert np.abs(q - q0).max() < 1e-14
    s.close()


def test_decay_gpu():
    case = make_case("C1_decay")
    s = Session(case)
    q0 = s.initial_state()
    s.set_state(q0)
    s.step(case.dt, 10)
    q, t, _ = s.get_state()
    exact = q0.copy()
    exact[:, 3:] = (q0[:, 3:] - case.extra["delta"]) + case.extra["delta"] * math.exp(-t / case.tau)
    assert np.abs(q - exact).max() < 1e-14
    s.close()


@pytest.mark.parametrize("N", [2, 3])
def test_sark_3d_few_steps_fp64(N):
    """3D moving Taylor-Green on 3^3 cubes x 6 tetrahedra: 4 SARK-4 steps at
    N = 2 and at the 3D workload's order N = 3."""
    case = make_case("C3", n=3, N=N)
    qg, o, t, step, xg = _run_both(case, 4)
    assert step == 4 and np.abs(xg - o.x).max() < 1e-14
    assert _rel(qg, o.q) < 1e-12


def test_sark_walled_ogrid_with_sponge_fp64():
    """Plunging O-grid with wall and far-field faces and the sponge: 20 SARK-4
    steps of the GPU FP64 path against the oracle (stand-ins, parity against
    the oracle's own definitions)."""
    vx, etov, per, tag = ogrid_airfoil(6, 24, radius=6.0)
    case = make_case("C4", N=3)
    case.vx, case.etov, case.period, case.face_tag = vx, etov, per, tag
    case.motion = dict(case.motion, r_in=1.0, r_out=4.0, omega=2.0)
    case.dt = cfl_dt(vx, etov, 3, 1.0, 0.3)
    q_inf = gb.equilibrium(2, np.array(1.0), [np.array(0.1), np.array(0.0)], 1.0)
    sponge = (0.5, 0.0, 4.5, 6.0, 2.0)
    s = Session(case, q_inf=q_inf, sponge=sponge)
    o = _oracle_for(case, q_inf=q_inf, sponge=sponge)
    q0 = _state(o, case)
    s.set_state(q0)
    o.set_state(q0)
    s.step(case.dt, 20)
    o.run(case.dt, 20)
    qg, t, step = s.get_state()
    assert step == 20
    assert _rel(qg, o.q) < 1e-12
    s.close()


def test_fp32_velocity_short_run():
    """FP32 with perturbation storage against the FP64 oracle: velocity
    within 1e-5 relative after 200 steps of the 32x32 copy of the 2D TGV."""
    case = make_case("C2_small")
    qg, o, *_ = _run_both(case, 200, precision=L.GB_FP32)
    ug = gb.velocity(2, qg.transpose(1, 0, 2), case.c)
    uo = gb.velocity(2, o.q.transpose(1, 0, 2), case.c)
    assert np.linalg.norm(ug - uo) / np.linalg.norm(uo) < 1e-5


def test_error_latch_nonphysical():
    """A non-positive density set from the host is latched by the kernel and
    reported by the next synchronising call."""
    case = make_case("C1", n=4)
    s = Session(case)
    q = s.initial_state()
    q[0, 0, :] = -1.0
    s.set_state(q)
    s.step(case.dt, 1)
    with pytest.raises(L.GbError) as ei:
        s.get_state()
    assert ei.value.status == L.GB_ERR_NONPHYSICAL
    s.close()


def test_vertex_array_motion_matches_analytic():
    """Grid velocities supplied per step at the four stage times (evaluated
    here by the oracle's motion) reproduce the analytic sin-product motion
    to rounding."""
    case = make_case("C1", n=8)
    s_a, s_v = Session(case), Session(case)
    q0 = s_a.initial_state()
    s_a.set_state(q0)
    s_v.set_state(q0)
    mot = dict(case.motion)
    om = Motion(mot.pop("kind"), **mot)
    X = np.asarray(case.vx, float)
    t = 0.0
    for _ in range(5):
        w4 = np.stack([om.velocity(X, t + c * case.dt) for c in (0.0, 0.5, 0.5, 1.0)])
        L.gb_set_vertex_velocity(s_v.mesh, w4)
        s_v.step(case.dt, 1)
        t += case.dt
    s_a.step(case.dt, 5)
    qa, ta, na = s_a.get_state()
    qv, tv, nv = s_v.get_state()
    assert na == nv == 5 and abs(ta - tv) < 1e-15
    assert _rel(qv, qa) < 1e-13
    with pytest.raises(L.GbError):
        L.gb_set_motion(s_v.mesh, L.GB_MOTION_VERTEX_ARRAY, [])
    s_a.close()
    s_v.close()
