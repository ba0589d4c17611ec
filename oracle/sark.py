"""Semi-analytic Runge-Kutta (SARK-4) coefficients and update (oracle).

Test infrastructure only (see ``oracle/__init__``).

Section 4 of the paper: dq/dt = -Lambda q + F(q) (eq. time_split) is advanced by
  q_ni    = exp(-Lambda dt_i) q_n + dt sum_{j<i} atilde_ij F_nj
  q_{n+1} = exp(-Lambda dt) q_n   + dt sum_j   btilde_j  F_nj
with stage times c = (0, 1/2, 1/2, 1) of the classical RK4 tableau
(table Butcher) and the closed-form coefficients printed in that section as
functions of gamma = -dt/tau.  The final sum runs over F_nj (the printed F_ni
is read as a typo).

The closed forms cancel catastrophically for small |gamma| and are singular at
gamma = 0; the oracle evaluates exactly those printed formulas in 50-digit
arithmetic (mpmath, with the working precision raised by the digits the
cancellation costs) and rounds once, and takes gamma = 0 (fields with no
relaxation) from the RK4 tableau, the limit the paper states the method
reduces to.
"""
from __future__ import annotations

import numpy as np
import mpmath as mp

C_STAGE = (0.0, 0.5, 0.5, 1.0)
RK4_A = {(1, 0): 0.5, (2, 0): 0.0, (2, 1): 0.5, (3, 0): 0.0, (3, 1): 0.0, (3, 2): 1.0}
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


def coefficients(gamma: float):
    """(atilde dict {(i,j): value}, btilde tuple) for gamma = -dt/tau."""
    if gamma == 0.0:
        return dict(RK4_A), tuple(RK4_B)
    # the btilde numerators cancel down to O(gamma^3): carry enough digits to
    # keep ~30 significant ones after the cancellation
    lost = max(0.0, -3.0 * mp.log10(abs(gamma)))
    with mp.workdps(int(40 + lost)):
        g = mp.mpf(gamma)
        eh, e1 = mp.exp(g / 2), mp.exp(g)
        a = {
            (1, 0): (-1 + eh) / g,
            (2, 0): (4 + g + eh * (g - 4)) / g**2,
            (2, 1): (-4 - 2 * g + 4 * eh) / g**2,
            (3, 0): (2 + g + e1 * (g - 2)) / g**2,
            (3, 1): mp.mpf(0),
            (3, 2): (-2 - 2 * g + 2 * e1) / g**2,
        }
        b = (
            (-4 - g + e1 * (g**2 - 3 * g + 4)) / g**3,
            (4 + 2 * g + e1 * (2 * g - 4)) / g**3,
            (4 + 2 * g + e1 * (2 * g - 4)) / g**3,
            (-4 - 3 * g - g**2 + e1 * (4 - g)) / g**3,
        )
        return {k: float(v) for k, v in a.items()}, tuple(float(v) for v in b)


def stage_decay(gamma: float, i: int) -> float:
    """exp(-Lambda dt_i) = exp(c_i gamma) for stage i (i = 4 is the final)."""
    c = 1.0 if i >= 3 else C_STAGE[i]
    with mp.workdps(50):
        return float(mp.exp(c * mp.mpf(gamma)))


class FieldCoefficients:
    """Per-field SARK coefficients: fields with rate 0 use RK4, the rest use
    gamma = -dt * rate."""

    def __init__(self, rates: np.ndarray, dt: float):
        nf = rates.size
        self.a = {k: np.zeros(nf) for k in RK4_A}
        self.b = np.zeros((4, nf))
        self.E = np.zeros((5, nf))   # E[i] multiplies q_n in stage i (i=4: final)
        for f in range(nf):
            g = -dt * rates[f]
            a, b = coefficients(g)
            for k in a:
                self.a[k][f] = a[k]
            self.b[:, f] = b
            for i in range(5):
                self.E[i, f] = stage_decay(g, i)
