"""Fourier pseudo-spectral reference for the continuous 2D Galerkin-Boltzmann
system on the periodic square [-1,1]^2 (Eulerian frame).

A textbook method independent of the DG oracle: spectral derivatives by FFT,
the collision term evaluated pointwise, and scipy's adaptive DOP853 in time.
It solves dq/dt = A_x q_x + A_y q_y + N(q) with the matrices and collision
operator printed in Section 2 of the paper (A_d = -sqrt(RT) M_d).
"""
import math

import numpy as np
from scipy.integrate import solve_ivp

S2 = math.sqrt(2.0)
# rows of A_x / (-sqrt(RT)) and A_y / (-sqrt(RT)) as printed
_MX = np.array([[0, 1, 0, 0, 0, 0], [1, 0, 0, 0, S2, 0], [0, 0, 0, 1, 0, 0],
                [0, 0, 1, 0, 0, 0], [0, S2, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0]], float)
_MY = np.array([[0, 0, 1, 0, 0, 0], [0, 0, 0, 1, 0, 0], [1, 0, 0, 0, 0, S2],
                [0, 1, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0], [0, 0, S2, 0, 0, 0]], float)


class Spectral2D:
    def __init__(self, n: int, c: float, tau: float):
        self.n, self.c, self.tau = n, c, tau
        self.x = -1.0 + 2.0 * np.arange(n) / n
        k = np.fft.fftfreq(n, d=1.0 / n) * math.pi       # wavenumbers pi * integer
        self.kx = k[None, :]                              # axis 1 is x
        self.ky = k[:, None]                              # axis 0 is y

    def rhs(self, t, y):
        n = self.n
        q = y.reshape(6, n, n)
        qh = np.fft.fft2(q)
        qx = np.real(np.fft.ifft2(1j * self.kx * qh))
        qy = np.real(np.fft.ifft2(1j * self.ky * qh))
        d = -self.c * (np.einsum("gf,fij->gij", _MX, qx) + np.einsum("gf,fij->gij", _MY, qy))
        r = q[0]
        coll = np.zeros_like(q)
        coll[3] = -(q[3] - q[1] * q[2] / r) / self.tau
        coll[4] = -(q[4] - q[1] ** 2 / (S2 * r)) / self.tau
        coll[5] = -(q[5] - q[2] ** 2 / (S2 * r)) / self.tau
        return (d + coll).ravel()

    def solve(self, q0, T):
        sol = solve_ivp(self.rhs, (0.0, T), q0.ravel(), method="DOP853", rtol=1e-12, atol=1e-14)
        assert sol.success
        return sol.y[:, -1].reshape(6, self.n, self.n)

    def evaluate(self, q, px, py):
        """Trigonometric interpolant of q [6, n, n] at points (px, py)."""
        n = self.n
        qh = np.fft.fft2(q) / (n * n)
        k = np.fft.fftfreq(n, d=1.0 / n)
        # e^{i pi k (x+1)} because grid starts at x=-1
        ex = np.exp(1j * math.pi * np.outer(px.ravel() + 1.0, k))   # [P, n] x-modes
        ey = np.exp(1j * math.pi * np.outer(py.ravel() + 1.0, k))   # [P, n] y-modes
        out = np.real(np.einsum("fab,pa,pb->fp", qh, ey, ex))
        return out.reshape((6,) + px.shape)
