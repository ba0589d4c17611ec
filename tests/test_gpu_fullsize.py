"""Parity at the workloads' full sizes, in the launch configuration bench.py
times, on sampled outputs the oracle computes one by one (one SARK-4 step
evaluated only on each sample's domain of dependence), and the FP32 accuracy
target over the full 2000-step run of the 32x32 copy of the 2D workload
against the oracle's stored solution (tests/golden/make_c2_small_reference.py).
"""
import os

import numpy as np
import pytest

from oracle import gbsystem as gb
from oracle.mesh import Mesh
from oracle.motion import Motion
from oracle.rhs import Params
from oracle.solver import Solver
from workloads import make_case

pytestmark = pytest.mark.gpu

from paper_2607_00199_amd import _lib as L  # noqa: E402
from paper_2607_00199_amd.session import Session  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_small_oracle_2000.npz")


def _oracle(case, **kw):
    mesh = Mesh(case.dim, case.N, case.vx, case.etov, case.period, face_tag=case.face_tag)
    mot = dict(case.motion)
    kind = mot.pop("kind")
    return Solver(mesh, Params(c=case.c, tau=case.tau, **kw), Motion(kind, **mot))


def _initial(o, case):
    X = o.node_coords()
    rho, u = case.macroscopic(X)
    return gb.equilibrium(case.dim, rho, u, case.c).transpose(1, 0, 2).copy()


def _sample(K, n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(K, n, replace=False), [0, 1, K - 2, K - 1]]))


def _check(qg, qo, rho_abs, rel):
    """Density within rho_abs absolute; momentum components within rel of the
    largest momentum component over the sample, stress components within rel
    of the largest stress component (a component that is ~0, such as m_z of
    the 3D vortex after one step, carries the rounding of its neighbours)."""
    dim = 2 if qo.shape[1] == 6 else 3
    assert np.abs(qg[:, 0] - qo[:, 0]).max() <= rho_abs
    groups = [range(1, dim + 1), range(dim + 1, qo.shape[1])]
    for grp in groups:
        scale = max(np.abs(qo[:, f]).max() for f in grp)
        for f in grp:
            assert np.abs(qg[:, f] - qo[:, f]).max() <= rel * scale, f


def _one_step_sampled(case, precision, extra_oracle=None, extra_session=None, nsamp=48, seed=0):
    o = _oracle(case, **(extra_oracle or {}))
    q0 = _initial(o, case)
    o.set_state(q0)
    s = Session(case, precision=precision, **(extra_session or {}))
    s.set_state(q0)
    s.step(case.dt, 1)
    qg, t, step = s.get_state()
    s.close()
    elems, qo = o.step_patch(case.dt, _sample(case.K, nsamp, seed))
    assert step == 1
    return qg[elems], qo


def test_c2_full_size_fp64_one_step():
    case = make_case("C2")
    qg, qo = _one_step_sampled(case, L.GB_FP64)
    _check(qg, qo, 1e-14, 1e-12)


def test_c2_full_size_fp32_one_step():
    case = make_case("C2")
    qg, qo = _one_step_sampled(case, L.GB_FP32)
    _check(qg, qo, 2e-7, 2e-5)


def test_c3_full_size_fp32_one_step():
    """3D moving Taylor-Green vortex, 663552 tetrahedra, N=3, FP32."""
    case = make_case("C3")
    qg, qo = _one_step_sampled(case, L.GB_FP32, nsamp=32)
    _check(qg, qo, 2e-7, 2e-5)


def test_c4_full_size_fp32_one_step():
    """Plunging-airfoil O-grid, 262144 triangles, N=4, FP32, walls, far field
    and sponge (stand-ins)."""
    case = make_case("C4")
    q_inf = gb.equilibrium(2, np.array(1.0), [np.array(case.extra["u"][0]), np.array(case.extra["u"][1])], case.c)
    sponge = case.extra["sponge"]
    qg, qo = _one_step_sampled(case, L.GB_FP32, {"q_inf": q_inf, "sponge": sponge},
                               {"q_inf": q_inf, "sponge": sponge})
    _check(qg, qo, 2e-7, 2e-5)


def test_fp32_velocity_2000_steps_vs_oracle():
    """FP32 with perturbation storage q1 - rho0 on the 32x32 copy of the 2D
    workload, 2000 SARK-4 steps: velocity within 1e-5 relative of the FP64
    oracle's stored solution."""
    ref = np.load(GOLDEN)
    case = make_case("C2_small")
    assert ref["K"] == case.K and ref["nsteps"] == case.nsteps and abs(float(ref["dt"]) - case.dt) < 1e-18
    s = Session(case, precision=L.GB_FP32)
    s.set_state(s.initial_state())
    s.step(case.dt, case.nsteps, graph=True)
    q, t, step = s.get_state()
    s.close()
    assert step == case.nsteps and abs(t - float(ref["t"])) < 1e-12
    u = np.stack([case.c * q[:, 1] / q[:, 0], case.c * q[:, 2] / q[:, 0]])
    uo = ref["velocity"]
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    assert err < 1e-5, err
