"""Workload definitions: the paper's test cases restated as seeded synthetic
inputs (mesh, order, physical parameters, motion, time step, step count).

Physical scaling: c = sqrt(RT) = 1, so the reference speed equals the Mach
number; nu = U L / Re and tau = nu / c^2 (Section 2: nu = tau RT).

Time step: dt = CFL * h_min / (c_max (N+1)^2) with h_min the smallest
inscribed diameter (4 area / perimeter in 2D, 6 volume / surface in 3D) and
c_max = sqrt(3) c + the largest grid speed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import fields, meshes


def inscribed_diameters(vx: np.ndarray, etov: np.ndarray) -> np.ndarray:
    P = vx[etov]
    dim = vx.shape[1]
    if dim == 2:
        a = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
        b = np.linalg.norm(P[:, 2] - P[:, 1], axis=1)
        c = np.linalg.norm(P[:, 0] - P[:, 2], axis=1)
        e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
        area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        return 4 * area / (a + b + c)
    e1, e2, e3 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]
    vol = np.abs(np.einsum("kd,kd->k", e1, np.cross(e2, e3))) / 6
    surf = 0.0
    for (i, j, k) in ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)):
        surf = surf + 0.5 * np.linalg.norm(np.cross(P[:, j] - P[:, i], P[:, k] - P[:, i]), axis=1)
    return 6 * vol / surf


def cfl_dt(vx, etov, N: int, c: float, wmax: float, cfl: float = 0.5) -> float:
    h = inscribed_diameters(vx, etov).min()
    return cfl * h / ((math.sqrt(3.0) * c + wmax) * (N + 1) ** 2)


@dataclass
class Case:
    name: str
    dim: int
    N: int
    vx: np.ndarray
    etov: np.ndarray
    period: np.ndarray
    face_tag: np.ndarray | None
    c: float
    tau: float
    motion: dict
    dt: float
    nsteps: int
    init: str                      # "tgv2d" | "tgv3d" | "uniform" | "decay"
    u0: float
    extra: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return self.etov.shape[0]

    def macroscopic(self, nodes_xyz: np.ndarray):
        """Initial (rho, u) at node coordinates [K, dim, Np]."""
        X = nodes_xyz
        if self.init == "tgv2d":
            return fields.taylor_green_2d(X[:, 0], X[:, 1], self.u0)
        if self.init == "tgv3d":
            return fields.taylor_green_3d(X[:, 0], X[:, 1], X[:, 2], self.u0, 1.0)
        if self.init in ("uniform", "decay"):
            u = self.extra.get("u", (self.u0,) * self.dim)
            return fields.uniform(X[:, 0].shape, 1.0, u)
        raise ValueError(self.init)


def _motion_speed(m: dict) -> float:
    k = m["kind"]
    if k == "none":
        return 0.0
    if k == "sin_product_2d":
        return math.hypot(*m["A"]) * 2 * math.pi / m["T"]
    if k == "triple_product_3d":
        return math.sqrt(3) * m["A"] * 2 * math.pi / m["T"]
    if k == "plunge_blend_2d":
        return m["h0"] * m["omega"]
    raise ValueError(k)


def make_case(name: str, **over) -> Case:
    """Build a named workload; keyword overrides replace defaults (e.g. n=32,
    N=3, nsteps=10, motion amplitude A=0)."""
    spec = dict(CASES[name])
    spec.update(over)
    kind = spec["mesh"]
    if kind == "square":
        vx, etov, period, tag = meshes.periodic_square(spec["n"], seed=spec.get("seed", 0),
                                                       jitter=spec.get("jitter", 0.05))
    elif kind == "kuhn":
        vx, etov, period, tag = meshes.kuhn_cube(spec["n"])
    elif kind == "ogrid":
        vx, etov, period, tag = meshes.ogrid_airfoil(spec["n_r"], spec["n_theta"])
    else:
        raise ValueError(kind)
    motion = dict(spec["motion"])
    c = spec["c"]
    nu = spec["u0"] * spec["Lref"] / spec["Re"]
    tau = nu / c**2
    dt = spec.get("dt") or cfl_dt(vx, etov, spec["N"], c, _motion_speed(motion) + spec["u0"],
                                  spec.get("cfl", 0.5))
    extra = {k: spec[k] for k in ("u", "delta", "sponge") if k in spec}
    return Case(name=name, dim=spec["dim"], N=spec["N"], vx=vx, etov=etov, period=period,
                face_tag=tag, c=c, tau=tau, motion=motion, dt=dt, nsteps=spec["nsteps"],
                init=spec["init"], u0=spec["u0"], extra=extra)


_SIN2D = {"kind": "sin_product_2d", "A": (0.05, 0.05), "T": 1.0, "L": (2.0, 2.0), "origin": (0.0, 0.0)}

CASES = {
    # 2D moving Taylor-Green vortex, 16x16 quads -> 512 triangles, N=3, FP64
    "C1": dict(mesh="square", n=16, dim=2, N=3, c=1.0, u0=0.1, Re=100.0, Lref=1 / math.pi,
               motion=_SIN2D, nsteps=200, init="tgv2d"),
    # free-stream variant on the same mesh and seed
    "C1_freestream": dict(mesh="square", n=16, dim=2, N=3, c=1.0, u0=0.1, Re=100.0, Lref=1 / math.pi,
                          motion=_SIN2D, nsteps=200, init="uniform", u=(0.1, 0.1)),
    # uniform non-equilibrium state: stresses off equilibrium by delta
    "C1_decay": dict(mesh="square", n=16, dim=2, N=3, c=1.0, u0=0.1, Re=100.0, Lref=1 / math.pi,
                     motion=_SIN2D, nsteps=200, init="decay", u=(0.1, 0.1), delta=1e-2),
    # 2D moving TGV at scale: 256x256 quads -> 131072 triangles, N=4
    "C2": dict(mesh="square", n=256, dim=2, N=4, c=1.0, u0=0.05, Re=1000.0, Lref=1 / math.pi,
               motion=_SIN2D, nsteps=2000, init="tgv2d"),
    # the 32x32 down-sized copy used for FP32-vs-oracle accuracy
    "C2_small": dict(mesh="square", n=32, dim=2, N=4, c=1.0, u0=0.05, Re=1000.0, Lref=1 / math.pi,
                     motion=_SIN2D, nsteps=2000, init="tgv2d"),
    # 3D moving TGV: 48^3 cubes x 6 Kuhn tets = 663552 tets, N=3
    "C3": dict(mesh="kuhn", n=48, dim=3, N=3, c=1.0, u0=0.1, Re=1600.0, Lref=1.0,
               motion={"kind": "triple_product_3d", "A": 0.03, "T": 20.0, "L": 2 * math.pi},
               nsteps=500, init="tgv3d"),
    # plunging NACA 0012 O-grid, 256 x 512 quads -> 262144 triangles, N=4;
    # the plunge frequency is in convective time (t U / chord): omega = 2 pi f U
    "C4": dict(mesh="ogrid", n_r=256, n_theta=512, dim=2, N=4, c=1.0, u0=0.1, Re=1e4, Lref=1.0,
               motion={"kind": "plunge_blend_2d", "h0": 0.1, "omega": 2 * math.pi * 0.5 * 0.1,
                       "r_in": 1.5, "r_out": 16.0, "center": (0.5, 0.0)},
               nsteps=5000, init="uniform", u=(0.1, 0.0),
               sponge=(0.5, 0.0, 16.0, 20.0, 2.0)),
}


def c5_requests(n: int = 64, seed: int = 1, mean_gap: float = 0.05, nsteps: int = 1000,
                sizes=(64, 128, 192, 256), orders=(2, 3, 4, 5)) -> list:
    """The served-request mix: n plunging-airfoil requests with exponential
    inter-arrival times (Poisson arrivals, mean gap in seconds), each with
    its own O-grid size (n_r radial layers, 2 n_r points around the body,
    K = 4 n_r^2 triangles), order, plunge amplitude h0 and frequency f, and
    Reynolds number; Mach 0.1, nsteps steps.  Drawn from
    numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap, size=n)
    arrival = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        n_r = int(rng.choice(sizes))
        out.append(dict(index=i, arrival=float(arrival[i]), n_r=n_r, n_theta=2 * n_r, N=int(rng.choice(orders)),
                        h0=float(rng.uniform(0.05, 0.2)), f=float(rng.uniform(0.25, 1.0)),
                        Re=float(rng.uniform(1e3, 1e4)), nsteps=nsteps))
    return out


def c5_case(req: dict) -> Case:
    """Case of one served request (the plunging-airfoil workload at the
    request's size, order and parameters)."""
    motion = dict(CASES["C4"]["motion"])
    # frequency f in convective time units (chord / U), U = 0.1
    motion.update(h0=req["h0"], omega=2 * math.pi * req["f"] * CASES["C4"]["u0"])
    return make_case("C4", n_r=req["n_r"], n_theta=req["n_theta"], N=req["N"], Re=req["Re"],
                     motion=motion, nsteps=req["nsteps"])