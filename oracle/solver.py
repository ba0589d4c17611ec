"""SARK-4 time stepping of the ALE scheme on a moving mesh (oracle).

Test infrastructure only (see ``oracle/__init__``).

Per step (Sections 4 and 5 of the paper):
  * vertex positions of the four RK4 stages and the end-of-step positions
    (``motion.stage_positions``); stage j is evaluated entirely on the
    geometry of its own positions with the grid velocity at its own time, so
    the geometric factors are rebuilt at every stage;
  * F_j = F(q_nj) at that geometry (``rhs.rhs``);
  * q_n1 = E(1/2) q_n + dt a10 F_0
    q_n2 = E(1/2) q_n + dt (a20 F_0 + a21 F_1)
    q_n3 = E(1)   q_n + dt (a30 F_0 + a31 F_1 + a32 F_2)
    q_n+1 = E(1)  q_n + dt (b0 F_0 + b1 F_1 + b2 F_2 + b3 F_3)
    field by field, E(c) = exp(-c dt rate), with the conserved fields on the
    RK4 limit of the coefficients.
"""
from __future__ import annotations

import numpy as np

from . import gbsystem as gb
from .motion import Motion, stage_positions
from .rhs import Params, element_geometry, rhs
from .sark import FieldCoefficients


class Solver:
    def __init__(self, mesh, prm: Params, motion: Motion | None = None):
        self.mesh, self.prm = mesh, prm
        self.motion = motion or Motion("none")
        self.X = mesh.vx.copy()          # reference (t = 0) vertex positions
        self.x = mesh.vx.copy()          # current vertex positions
        self.t = 0.0
        self.step_index = 0
        self.q = None
        self._coef = {}

    def set_state(self, q: np.ndarray, t0: float = 0.0):
        self.q = np.array(q, float, copy=True)
        self.t = float(t0)

    def node_coords(self) -> np.ndarray:
        """Current node coordinates [K, dim, Np]."""
        P = self.x[self.mesh.etov]
        return np.einsum("pv,kvd->kdp", self.mesh.ref.bary, P)

    def rhs_now(self, q=None) -> np.ndarray:
        """F at the current geometry and time (stage-0 grid velocity)."""
        w = self.motion.velocity(self.X, self.t)
        return rhs(self.mesh, self.prm, self.q if q is None else q, self.x, w)

    def coefficients(self, dt: float) -> FieldCoefficients:
        if dt not in self._coef:
            rates = gb.relaxation_rates(self.mesh.dim, self.prm.tau)
            self._coef[dt] = FieldCoefficients(rates, dt)
        return self._coef[dt]

    def step(self, dt: float):
        cf = self.coefficients(dt)
        xs, ws, x_next = stage_positions(self.motion, self.X, self.x, self.t, dt)
        qn = self.q
        E = lambda i: cf.E[i][None, :, None]
        a = {k: v[None, :, None] for k, v in cf.a.items()}
        b = [cf.b[j][None, :, None] for j in range(4)]
        F0 = rhs(self.mesh, self.prm, qn, xs[0], ws[0])
        q1 = E(1) * qn + dt * a[(1, 0)] * F0
        F1 = rhs(self.mesh, self.prm, q1, xs[1], ws[1])
        q2 = E(2) * qn + dt * (a[(2, 0)] * F0 + a[(2, 1)] * F1)
        F2 = rhs(self.mesh, self.prm, q2, xs[2], ws[2])
        q3 = E(3) * qn + dt * (a[(3, 0)] * F0 + a[(3, 1)] * F1 + a[(3, 2)] * F2)
        F3 = rhs(self.mesh, self.prm, q3, xs[3], ws[3])
        self.q = E(4) * qn + dt * (b[0] * F0 + b[1] * F1 + b[2] * F2 + b[3] * F3)
        self.x = x_next
        self.t += dt
        self.step_index += 1

    def step_patch(self, dt: float, elems) -> tuple:
        """One SARK-4 step from the current state, evaluated only on the
        domains of dependence of ``elems`` (each stage reaches one ring of face
        neighbours further): F_0 on the 3-ring, F_1 on the 2-ring, F_2 on the
        1-ring, F_3 on ``elems``.  Returns (sorted elems, q_{n+1} there).  The
        solver state is not changed."""
        mesh = self.mesh
        rings = [np.unique(np.asarray(elems, np.int64))]
        for _ in range(3):
            rings.append(mesh.neighbours(rings[-1]))
        R0, R1, R2, R3 = rings
        cf = self.coefficients(dt)
        xs, ws, _ = stage_positions(self.motion, self.X, self.x, self.t, dt)
        qn = self.q
        E = lambda i: cf.E[i][None, :, None]
        a = {k: v[None, :, None] for k, v in cf.a.items()}
        b = [cf.b[j][None, :, None] for j in range(4)]
        F0, F1, F2 = (np.zeros_like(qn) for _ in range(3))
        q1, q2, q3 = (np.zeros_like(qn) for _ in range(3))
        F0[R3] = rhs(mesh, self.prm, qn, xs[0], ws[0], R3)
        q1[R3] = E(1) * qn[R3] + dt * a[(1, 0)] * F0[R3]
        F1[R2] = rhs(mesh, self.prm, q1, xs[1], ws[1], R2)
        q2[R2] = E(2) * qn[R2] + dt * (a[(2, 0)] * F0[R2] + a[(2, 1)] * F1[R2])
        F2[R1] = rhs(mesh, self.prm, q2, xs[2], ws[2], R1)
        q3[R1] = E(3) * qn[R1] + dt * (a[(3, 0)] * F0[R1] + a[(3, 1)] * F1[R1] + a[(3, 2)] * F2[R1])
        F3 = rhs(mesh, self.prm, q3, xs[3], ws[3], R0)
        out = E(4) * qn[R0] + dt * (b[0] * F0[R0] + b[1] * F1[R0] + b[2] * F2[R0] + b[3] * F3)
        return R0, out

    def run(self, dt: float, nsteps: int):
        for _ in range(nsteps):
            self.step(dt)

    def integrals(self, q=None) -> np.ndarray:
        """Integral over the current mesh of each field, [NF]:
        sum_e J_e 1^T M q_e (reference mass matrix M, Section 3)."""
        q = self.q if q is None else q
        J = element_geometry(self.mesh, self.x, np.arange(self.mesh.K))[0]
        w = self.mesh.ref.M.sum(axis=0)                         # 1^T M
        return np.einsum("k,p,kfp->f", J, w, q)

    def l2_norm(self, v: np.ndarray) -> np.ndarray:
        """Mass-weighted L2 norm per field of v [K, NF, Np] on the current mesh."""
        J = element_geometry(self.mesh, self.x, np.arange(self.mesh.K))[0]
        Mv = np.einsum("ij,kfj->kfi", self.mesh.ref.M, v)
        return np.sqrt(np.einsum("k,kfi,kfi->f", J, v, Mv))
