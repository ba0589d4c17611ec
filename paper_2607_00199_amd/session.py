"""Convenience wrapper: one context + mesh + solver built from a workload.

Argument marshalling only; every step of the path runs in libgb.so.
"""
from __future__ import annotations

import numpy as np

from . import _lib as L


def motion_params(motion: dict):
    """gb_motion (kind, p[]) for a workload motion description."""
    k = motion["kind"]
    if k == "none":
        return L.GB_MOTION_NONE, []
    if k == "sin_product_2d":
        X0, Y0 = motion.get("origin", (0.0, 0.0))
        return L.GB_MOTION_SIN_PRODUCT_2D, [motion["A"][0], motion["A"][1], motion["T"],
                                             motion["L"][0], motion["L"][1], X0, Y0]
    if k == "triple_product_3d":
        return L.GB_MOTION_TRIPLE_PRODUCT_3D, [motion["A"], motion["T"], motion["L"]]
    if k == "plunge_blend_2d":
        cx, cy = motion.get("center", (0.0, 0.0))
        return L.GB_MOTION_PLUNGE_BLEND_2D, [motion["h0"], motion["omega"], motion["r_in"],
                                              motion["r_out"], cx, cy]
    if k == "fish_3d":
        return L.GB_MOTION_FISH_3D, [motion["a0"], motion["a1"], motion["a2"], motion["lam"], motion["f"],
                                     motion["R_rigid"], motion["beta"], motion["T_ramp"]]
    raise ValueError(k)


def equilibrium_moments(dim: int, rho, u, c: float) -> np.ndarray:
    """Moments [NF, ...] of the equilibrium state with density rho and
    velocity u (u[d] arrays of rho's shape), computed by the library."""
    rho = np.asarray(rho, float)
    q = L.gb_equilibrium_moments(dim, c, rho.ravel(), np.stack([np.asarray(u[d], float).ravel() for d in range(dim)]))
    return q.reshape((q.shape[0],) + rho.shape)


def initial_offset(case, NF: int):
    """Per-field offset added to the equilibrium moments (the uniform
    off-equilibrium stress of the decay case), or None."""
    if case.init != "decay":
        return None
    off = np.zeros(NF)
    off[case.dim + 1:] = case.extra["delta"]
    return off


class Session:
    """Context, mesh and solver for a ``workloads`` case."""

    def __init__(self, case, precision=L.GB_FP64, flux_mode=L.GB_FLUX_SPLIT, device=0, stream=0,
                 rho0=1.0, cubature_degree=0, q_inf=None, sponge=None):
        self.case = case
        self.dim, self.N = case.dim, case.N
        self.ctx = L.gb_ctx_create(device, stream)
        self.mesh = L.gb_mesh_create(self.ctx, case.dim, case.N, case.vx, case.etov, case.period, case.face_tag)
        kind, p = motion_params(case.motion)
        L.gb_set_motion(self.mesh, kind, p)
        self.K, self.Np, self.NF, self.Nfp, self.Nfaces = L.gb_mesh_sizes(self.mesh)
        self.params = L.make_params(case.c, case.tau, precision, flux_mode, rho0, cubature_degree, q_inf, sponge)
        self.solver = L.gb_solver_create(self.mesh, self.params)

    @property
    def shape(self):
        return (self.K, self.NF, self.Np)

    def nodes(self) -> np.ndarray:
        return L.gb_mesh_nodes(self.mesh, self.dim)

    def initial_state(self) -> np.ndarray:
        """Equilibrium moments of the case's initial macroscopic fields [K, NF, Np]."""
        rho, u = self.case.macroscopic(self.nodes())
        q = equilibrium_moments(self.dim, rho, u, self.case.c).transpose(1, 0, 2).copy()
        off = initial_offset(self.case, self.NF)
        if off is not None:
            q += off[None, :, None]
        return q

    def set_initial_state(self, t0=0.0):
        """The case's initial state, formed on the device from the macroscopic
        fields at the nodes (gb_state_set_equilibrium)."""
        rho, u = self.case.macroscopic(self.nodes())
        L.gb_state_set_equilibrium(self.solver, rho, np.stack(u, axis=1), initial_offset(self.case, self.NF), t0)

    def set_state(self, q, t0=0.0):
        L.gb_state_set(self.solver, q, t0)

    def energy(self, rho_inf=1.0):
        """(E_K, epsilon_1, volume) at the current state."""
        return L.gb_energy(self.solver, rho_inf)

    def wall_force(self):
        """(pressure force, viscous force) on the wall faces."""
        return L.gb_wall_force(self.solver, self.dim)

    def checkpoint(self) -> bytes:
        return L.gb_checkpoint_save(self.solver)

    def restore(self, data: bytes):
        L.gb_checkpoint_load(self.solver, data)

    def get_state(self):
        return L.gb_state_get(self.solver, self.shape)

    def rhs(self, q):
        return L.gb_rhs(self.solver, q)

    def step(self, dt, n, graph=False):
        (L.gb_sark_step_graph if graph else L.gb_sark_step)(self.solver, dt, n)

    def close(self):
        if self.solver:
            L.gb_solver_destroy(self.solver)
            L.gb_mesh_destroy(self.mesh)
            L.gb_ctx_destroy(self.ctx)
            self.solver = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
