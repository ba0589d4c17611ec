"""Prescribed mesh motions and the RK4 vertex update (oracle).

Test infrastructure only (see ``oracle/__init__``).

Section 5 of the paper: the grid velocity is prescribed at the mesh vertices
and interpolated linearly (continuous P1) so elements stay affine; vertex
coordinates are advanced with the same Runge-Kutta scheme as the solution
(classical RK4, table Butcher), solving dx/dt = v_G with v_G the time
derivative of the prescribed displacement at fixed reference position X.

Motion kinds (displacement d(X, t), x = X + d):
  * "none";
  * "sin_product_2d" -- eq. gcl_exact_field:
      d = (Ax, Ay) sin(2 pi t/T) sin(2 pi (X-X0)/Lx) sin(2 pi (Y-Y0)/Ly);
  * "triple_product_3d" -- eq. TGV_deformation:
      d_x = A sin(2 pi t/T) sin(2 pi (Y+L/2)/L) sin(2 pi (Z+L/2)/L), and cyclic;
  * "plunge_blend_2d" -- the plunge y = Y - h0 sin(omega t) of Section 7.3,
      multiplied by a radial weight B(|X - centre|) that is 1 inside r_in and
      falls to 0 at r_out by a cosine ramp (the weight is a choice made here so
      the outer boundary stays fixed: the paper moves the whole grid rigidly);
  * "fish_3d" -- the carangiform swimming motion of Section 7.4 (eq.
      fish_motion, eq. fish_amplitude_function and the blended mesh motion
      that follows them), lengths in body lengths L = 1: only z moves,
        d_z = A(xt) sin(phi) B(d_eff) S(t),
        xt = min(1, max(0, X)),  A(xt) = a0 + a1 xt + a2 xt^2,
        phi = 2 pi X / lam - 2 pi f t,
        d_eff = max(|(X - xt, Y, Z)| - R_rigid, 0),  B = exp(-beta d_eff^2),
        S = (1 - cos(pi t / T_ramp)) / 2 for t < T_ramp, else 1.
      The paper prints the displacement with a factor "R" where the ramp S
      belongs (its printed mesh velocity is the time derivative of the form
      above); T_ramp <= 0 means no ramp.
"""
from __future__ import annotations

import math

import numpy as np


class Motion:
    def __init__(self, kind: str = "none", **p):
        self.kind = kind
        self.p = p

    def displacement(self, X: np.ndarray, t: float) -> np.ndarray:
        return self._eval(X, t, deriv=False)

    def velocity(self, X: np.ndarray, t: float) -> np.ndarray:
        """v_G(X, t) = d/dt displacement, [nv, dim]."""
        return self._eval(X, t, deriv=True)

    def _eval(self, X, t, deriv):
        X = np.asarray(X, float)
        out = np.zeros_like(X)
        p = self.p
        k = self.kind
        if k == "none":
            return out
        if k == "sin_product_2d":
            om = 2 * math.pi / p["T"]
            tt = om * math.cos(om * t) if deriv else math.sin(om * t)
            X0, Y0 = p.get("origin", (0.0, 0.0))
            sp = (np.sin(2 * math.pi * (X[:, 0] - X0) / p["L"][0])
                  * np.sin(2 * math.pi * (X[:, 1] - Y0) / p["L"][1]))
            out[:, 0] = p["A"][0] * tt * sp
            out[:, 1] = p["A"][1] * tt * sp
            return out
        if k == "triple_product_3d":
            om = 2 * math.pi / p["T"]
            tt = om * math.cos(om * t) if deriv else math.sin(om * t)
            L = p["L"]
            s = [np.sin(2 * math.pi * (X[:, d] + L / 2) / L) for d in range(3)]
            out[:, 0] = p["A"] * tt * s[1] * s[2]
            out[:, 1] = p["A"] * tt * s[0] * s[2]
            out[:, 2] = p["A"] * tt * s[0] * s[1]
            return out
        if k == "plunge_blend_2d":
            om = p["omega"]
            tt = om * math.cos(om * t) if deriv else math.sin(om * t)
            cx, cy = p.get("center", (0.0, 0.0))
            r = np.hypot(X[:, 0] - cx, X[:, 1] - cy)
            r0, r1 = p["r_in"], p["r_out"]
            xi = np.clip((r - r0) / (r1 - r0), 0.0, 1.0)
            B = 0.5 * (1.0 + np.cos(math.pi * xi))
            out[:, 1] = -p["h0"] * tt * B
            return out
        if k == "fish_3d":
            xt = np.clip(X[:, 0], 0.0, 1.0)
            amp = p["a0"] + p["a1"] * xt + p["a2"] * xt * xt
            om = 2 * math.pi * p["f"]
            phi = 2 * math.pi * X[:, 0] / p["lam"] - om * t
            dist = np.sqrt((X[:, 0] - xt) ** 2 + X[:, 1] ** 2 + X[:, 2] ** 2)
            d_eff = np.maximum(dist - p["R_rigid"], 0.0)
            B = np.exp(-p["beta"] * d_eff ** 2)
            Tr = p["T_ramp"]
            if Tr > 0 and t < Tr:
                S = 0.5 * (1.0 - math.cos(math.pi * t / Tr))
                dS = 0.5 * math.pi / Tr * math.sin(math.pi * t / Tr)
            else:
                S, dS = 1.0, 0.0
            if deriv:
                out[:, 2] = amp * B * (-om * np.cos(phi) * S + np.sin(phi) * dS)
            else:
                out[:, 2] = amp * np.sin(phi) * B * S
            return out
        raise ValueError(f"unknown motion kind {k!r}")


def stage_positions(motion: Motion, X: np.ndarray, x_n: np.ndarray, t_n: float, dt: float):
    """Vertex positions x_nj and vertex velocities w_j at the four RK4 stages,
    and the end-of-step positions x_{n+1}.  The right-hand side of the vertex
    ODE depends only on (X, t), so the RK4 stage slopes are the velocities at
    the stage times t_n + c_j dt."""
    w = [motion.velocity(X, t_n + c * dt) for c in (0.0, 0.5, 0.5, 1.0)]
    x = [x_n,
         x_n + 0.5 * dt * w[0],
         x_n + 0.5 * dt * w[1],
         x_n + dt * w[2]]
    x_next = x_n + dt * (w[0] + 2 * w[1] + 2 * w[2] + w[3]) / 6.0
    return x, w, x_next
