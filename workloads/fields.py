"""Closed-form initial fields in macroscopic variables (density, velocity)."""
from __future__ import annotations

import math

import numpy as np


def taylor_green_2d(x: np.ndarray, y: np.ndarray, u0: float):
    """2D Taylor-Green vortex on [-1,1]^2 with uniform density 1:
    u = u0 sin(pi x) cos(pi y), v = -u0 cos(pi x) sin(pi y)."""
    rho = np.ones_like(x)
    u = u0 * np.sin(math.pi * x) * np.cos(math.pi * y)
    v = -u0 * np.cos(math.pi * x) * np.sin(math.pi * y)
    return rho, (u, v)


def taylor_green_3d(x, y, z, U0: float, L: float = 1.0):
    """3D Taylor-Green vortex (Section 7.2 initial state) with uniform density 1:
    u = U0 sin(x/L) cos(y/L) cos(z/L), v = -U0 cos(x/L) sin(y/L) cos(z/L), w = 0."""
    rho = np.ones_like(x)
    u = U0 * np.sin(x / L) * np.cos(y / L) * np.cos(z / L)
    v = -U0 * np.cos(x / L) * np.sin(y / L) * np.cos(z / L)
    return rho, (u, v, np.zeros_like(x))


def uniform(shape, rho: float, u):
    """Spatially uniform state."""
    return np.full(shape, rho), tuple(np.full(shape, ud) for ud in u)
