"""Galerkin-Boltzmann moment system (oracle).

Test infrastructure only (see ``oracle/__init__``).

2D: Section 2 of the paper -- the six-field system dq/dt = A_x dq/dx +
A_y dq/dy + N(q) (eq. stationary_bns) with A_d = -sqrt(RT) M_d, M_d the
printed 0/1/sqrt(2) patterns, and the collision operator N(q).  The time split
of Section 4 (eq. time_split) writes N(q) = -Lambda q + Ntilde(q) with
Lambda = diag(0,0,0,1/tau,1/tau,1/tau).

3D: the paper prints no 3D matrices (it only cites them).  The oracle uses the
tensor form that reproduces the printed 2D system exactly when the z-parts are
dropped:  rho_t = -c div m,  m_t = -c div(rho I + S),
S_t = -c (grad m + grad m^T) - (S - m m^T / rho)/tau, with fields
(rho, m_x, m_y, m_z, S_xy, S_xz, S_yz, S_xx/sqrt2, S_yy/sqrt2, S_zz/sqrt2).
Parity unpinned against the paper for the 3D system.

``c`` denotes sqrt(RT) throughout.
"""
from __future__ import annotations

import math

import numpy as np

SQ2 = math.sqrt(2.0)


def n_fields(dim: int) -> int:
    return 6 if dim == 2 else 10


def n_conserved(dim: int) -> int:
    """Fields with zero relaxation rate: density and momentum."""
    return dim + 1


def flux_patterns(dim: int):
    """The matrices M_d with A_d = -c M_d (Section 2)."""
    if dim == 2:
        Mx = np.zeros((6, 6))
        My = np.zeros((6, 6))
        # printed A_x / (-sqrt(RT)), rows 1..6
        Mx[0, 1] = 1
        Mx[1, 0] = 1
        Mx[1, 4] = SQ2
        Mx[2, 3] = 1
        Mx[3, 2] = 1
        Mx[4, 1] = SQ2
        # printed A_y / (-sqrt(RT))
        My[0, 2] = 1
        My[1, 3] = 1
        My[2, 0] = 1
        My[2, 5] = SQ2
        My[3, 1] = 1
        My[5, 2] = SQ2
        return [Mx, My]
    # 3D tensor form; index maps
    RHO, M = 0, (1, 2, 3)
    OFF = {(0, 1): 4, (1, 0): 4, (0, 2): 5, (2, 0): 5, (1, 2): 6, (2, 1): 6}
    DIAG = (7, 8, 9)
    mats = []
    for d in range(3):
        A = np.zeros((10, 10))
        # rho_t = -c d_d m_d
        A[RHO, M[d]] = 1.0
        # m_i,t = -c d_d (rho delta_id + S_id)
        A[M[d], RHO] += 1.0
        for i in range(3):
            if i == d:
                A[M[i], DIAG[i]] += SQ2          # S_ii = sqrt2 * q_diag
            else:
                A[M[i], OFF[(i, d)]] += 1.0
        # S_ij,t = -c (d_i m_j + d_j m_i); stored S_ij (i != j) and S_ii/sqrt2
        for i in range(3):
            for j in range(i + 1, 3):
                if d == i:
                    A[OFF[(i, j)], M[j]] += 1.0
                if d == j:
                    A[OFF[(i, j)], M[i]] += 1.0
            if d == i:
                A[DIAG[i], M[i]] += SQ2           # (S_ii/sqrt2)_t = -(2/sqrt2) c d_i m_i
        mats.append(A)
    return mats


def relaxation_rates(dim: int, tau: float) -> np.ndarray:
    """Diagonal of Lambda (eq. time_split)."""
    lam = np.zeros(n_fields(dim))
    lam[n_conserved(dim):] = 1.0 / tau
    return lam


def ntilde(dim: int, q: np.ndarray, tau: float) -> np.ndarray:
    """Nonlinear part Ntilde(q) of the collision operator (Section 4).

    q has the field index first: q[f, ...].  Returns an array of the same shape
    with zeros in the conserved fields.
    """
    out = np.zeros_like(q)
    rho = q[0]
    if dim == 2:
        mx, my = q[1], q[2]
        out[3] = mx * my / (tau * rho)
        out[4] = mx * mx / (SQ2 * tau * rho)
        out[5] = my * my / (SQ2 * tau * rho)
        return out
    mx, my, mz = q[1], q[2], q[3]
    out[4] = mx * my / (tau * rho)
    out[5] = mx * mz / (tau * rho)
    out[6] = my * mz / (tau * rho)
    out[7] = mx * mx / (SQ2 * tau * rho)
    out[8] = my * my / (SQ2 * tau * rho)
    out[9] = mz * mz / (SQ2 * tau * rho)
    return out


def collision(dim: int, q: np.ndarray, tau: float) -> np.ndarray:
    """N(q) = -Lambda q + Ntilde(q)."""
    lam = relaxation_rates(dim, tau)
    shape = (-1,) + (1,) * (q.ndim - 1)
    return -lam.reshape(shape) * q + ntilde(dim, q, tau)


def equilibrium(dim: int, rho, u, c: float) -> np.ndarray:
    """Moments of the equilibrium state with density rho and velocity u
    (u[d] arrays): rho u = c q_momentum (Section 2), stresses at N(q)=0."""
    rho = np.asarray(rho, float)
    m = [rho * np.asarray(u[d], float) / c for d in range(dim)]
    q = np.zeros((n_fields(dim),) + rho.shape)
    q[0] = rho
    for d in range(dim):
        q[1 + d] = m[d]
    # Ntilde*tau gives exactly the stress values at which N vanishes
    q += ntilde(dim, q, 1.0)
    return q


def velocity(dim: int, q: np.ndarray, c: float) -> np.ndarray:
    """Macroscopic velocity u_d = c q_{1+d} / q_0 (Section 2)."""
    return np.stack([c * q[1 + d] / q[0] for d in range(dim)])
