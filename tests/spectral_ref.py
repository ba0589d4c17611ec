"""Fourier pseudo-spectral references for the continuous Galerkin-Boltzmann
systems on periodic boxes (Eulerian frame): the 2D system on [-1,1]^2 and the
3D system on [-pi,pi]^3.

A textbook method independent of the DG oracle: spectral derivatives by FFT,
the collision term evaluated pointwise, and scipy's adaptive DOP853 in time.
The 2D one solves dq/dt = A_x q_x + A_y q_y + N(q) with the matrices and
collision operator printed in Section 2 of the paper (A_d = -sqrt(RT) M_d).
The 3D one is written from the tensor form of the moment system, without flux
matrices: rho_t = -c div m, m_t = -c div(rho I + S),
S_t = -c (grad m + grad m^T) - (S - m m^T / rho) / tau, with the fields
(rho, m_x, m_y, m_z, S_xy, S_xz, S_yz, S_xx/sqrt2, S_yy/sqrt2, S_zz/sqrt2).
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


class Spectral3D:
    def __init__(self, n: int, c: float, tau: float):
        self.n, self.c, self.tau = n, c, tau
        self.x = -math.pi + 2.0 * math.pi * np.arange(n) / n
        k = np.fft.fftfreq(n, d=1.0 / n)                  # integer wavenumbers on [-pi, pi]
        # array axes (z, y, x)
        self.k = [k[None, None, :], k[None, :, None], k[:, None, None]]

    def _d(self, f, a):
        return np.real(np.fft.ifftn(1j * self.k[a] * np.fft.fftn(f)))

    def rhs(self, t, y):
        n, c, tau = self.n, self.c, self.tau
        q = y.reshape(10, n, n, n)
        rho, m = q[0], q[1:4]
        S = np.empty((3, 3, n, n, n))
        off = {(0, 1): 4, (0, 2): 5, (1, 2): 6}
        for (a, b), i in off.items():
            S[a, b] = S[b, a] = q[i]
        for a in range(3):
            S[a, a] = S2 * q[7 + a]
        out = np.empty_like(q)
        dm = [[self._d(m[b], a) for b in range(3)] for a in range(3)]     # dm[a][b] = d_a m_b
        out[0] = -c * (dm[0][0] + dm[1][1] + dm[2][2])
        for a in range(3):
            out[1 + a] = -c * (self._d(rho, a) + sum(self._d(S[a, b], b) for b in range(3)))
        for (a, b), i in off.items():
            out[i] = -c * (dm[a][b] + dm[b][a]) - (S[a, b] - m[a] * m[b] / rho) / tau
        for a in range(3):
            out[7 + a] = (-c * 2.0 * dm[a][a] - (S[a, a] - m[a] * m[a] / rho) / tau) / S2
        return out.ravel()

    def solve(self, q0, T):
        sol = solve_ivp(self.rhs, (0.0, T), q0.ravel(), method="DOP853", rtol=1e-11, atol=1e-13)
        assert sol.success
        return sol.y[:, -1].reshape((10,) + (self.n,) * 3)

    def evaluate(self, q, px, py, pz):
        """Trigonometric interpolant of q [10, n, n, n] at points (px, py, pz)."""
        n = self.n
        qh = np.fft.fftn(q, axes=(1, 2, 3)) / n ** 3
        k = np.fft.fftfreq(n, d=1.0 / n)
        P = px.size
        out = np.empty((10, P))
        for s in range(0, P, 1024):                       # points in chunks: x, then y, then z
            sl = slice(s, min(P, s + 1024))
            ex = np.exp(1j * np.outer(px.ravel()[sl] + math.pi, k))
            ey = np.exp(1j * np.outer(py.ravel()[sl] + math.pi, k))
            ez = np.exp(1j * np.outer(pz.ravel()[sl] + math.pi, k))
            t1 = np.einsum("fcba,pa->fcbp", qh, ex)
            t2 = np.einsum("fcbp,pb->fcp", t1, ey)
            out[:, sl] = np.real(np.einsum("fcp,pc->fp", t2, ez))
        return out.reshape((10,) + px.shape)
