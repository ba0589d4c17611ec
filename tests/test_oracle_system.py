"""Pins for the oracle's moment system and SARK-4 coefficients."""
import math

import numpy as np
import pytest

from oracle import gbsystem as gb
from oracle import sark


# ---------------------------------------------------------------- moment system

def _Mn(dim, n):
    return sum(n[d] * M for d, M in enumerate(gb.flux_patterns(dim)))


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, 2.5, 4.0])
def test_2d_normal_flux_spectrum(theta):
    """The 2D system is hyperbolic with characteristic speeds c*{+-sqrt3, +-1,
    0, 0} in every direction (the symmetric 0/1/sqrt2 patterns of Section 2)."""
    n = (math.cos(theta), math.sin(theta))
    Mn = _Mn(2, n)
    assert np.allclose(Mn, Mn.T)
    ev = np.sort(np.linalg.eigvalsh(Mn))
    assert np.allclose(ev, [-math.sqrt(3), -1, 0, 0, 1, math.sqrt(3)], atol=1e-14)


def test_3d_normal_flux_spectrum():
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        Mn = _Mn(3, n)
        assert np.allclose(Mn, Mn.T)
        ev = np.sort(np.linalg.eigvalsh(Mn))
        assert np.allclose(ev, [-math.sqrt(3), -1, -1, 0, 0, 0, 0, 1, 1, math.sqrt(3)], atol=1e-13)


def test_3d_system_restricts_to_2d():
    """Dropping z (fields m_z, S_xz, S_yz, S_zz and the z-derivative) from the
    3D tensor system gives back the printed 2D system field for field."""
    keep = [0, 1, 2, 4, 7, 8]
    M3 = gb.flux_patterns(3)
    M2 = gb.flux_patterns(2)
    for d in range(2):
        assert np.array_equal(M3[d][np.ix_(keep, keep)], M2[d])
        # and the z-coupled fields never feed the kept ones through x or y
        others = [i for i in range(10) if i not in keep]
        assert np.all(M3[d][np.ix_(keep, others)] == 0)
    rng = np.random.default_rng(0)
    q3 = rng.uniform(0.5, 1.5, size=(10, 7))
    q3[3] = 0.0      # m_z = 0
    nt3 = gb.ntilde(3, q3, 0.7)
    nt2 = gb.ntilde(2, q3[keep], 0.7)
    assert np.allclose(nt3[keep], nt2)


def test_macroscopic_conservation_laws():
    """rho_t = -div(rho u) and the momentum equation carries grad p with
    p = rho RT (Section 2): with rho u = c q2, the q1 row of A_x is -c e2 and
    the q2 row has -c in the q1 column (pressure gradient / c)."""
    c = 0.37
    Mx, My = gb.flux_patterns(2)
    Ax, Ay = -c * Mx, -c * My
    # d rho/dt = Ax[0].q_x + Ay[0].q_y = -c (q2_x + q3_y) = -div(rho u)
    assert np.array_equal(Ax[0], -c * np.eye(6)[1])
    assert np.array_equal(Ay[0], -c * np.eye(6)[2])
    # d(rho u)/dt = c d q2/dt contains -c^2 d rho/dx = -RT d rho/dx = -dp/dx
    assert Ax[1, 0] * c == pytest.approx(-c * c)
    assert Ay[2, 0] * c == pytest.approx(-c * c)


def test_equilibrium_zero_collision_and_stress():
    """N(q) vanishes at equilibrium and the deviatoric stress of Section 2 is
    zero there."""
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.8, 1.2, 20)
    u = rng.uniform(-0.1, 0.1, (2, 20))
    c = 1.3
    q = gb.equilibrium(2, rho, u, c)
    assert np.abs(gb.collision(2, q, 0.01)).max() < 1e-15 / 0.01 * 10
    RT = c * c
    s11 = -RT * (math.sqrt(2) * q[4] - q[1] ** 2 / q[0])
    s22 = -RT * (math.sqrt(2) * q[5] - q[2] ** 2 / q[0])
    s12 = -RT * (q[3] - q[1] * q[2] / q[0])
    assert np.abs(np.stack([s11, s22, s12])).max() < 1e-15
    assert np.allclose(gb.velocity(2, q, c), u)


# ---------------------------------------------------------------- SARK-4

def test_sark_limit_is_rk4():
    """The method reduces to the base RK4 tableau (table Butcher) as
    1/tau -> 0."""
    for g in (-1e-6, -1e-9):
        a, b = sark.coefficients(g)
        for k, v in sark.RK4_A.items():
            assert abs(a[k] - v) < 1e-5 * 10 * abs(g) / 1e-6
        assert np.allclose(b, sark.RK4_B, atol=2e-6)


@pytest.mark.parametrize("g", [-1e-8, -1e-3, -0.5, -2.0, -20.0, -1e3])
def test_sark_row_sums(g):
    """eq. sark_coefficient_sum: sum_j b_j = (e^g - 1)/g, and the stage rows
    sum to (e^{c_i g} - 1)/g (the printed extra 1/c_i is read as a typo: the
    printed atilde_10 itself satisfies the version without it)."""
    a, b = sark.coefficients(g)
    import mpmath as mp
    with mp.workdps(40):
        G = mp.mpf(g)
        phi = lambda c: float((mp.exp(c * G) - 1) / G)
        assert abs(sum(b) - phi(1.0)) < 1e-15
        for i, ci in ((1, 0.5), (2, 0.5), (3, 1.0)):
            s = sum(v for (ii, j), v in a.items() if ii == i)
            assert abs(s - phi(ci)) < 1e-15


@pytest.mark.parametrize("g", [-1e-3, -0.5, -3.0, -50.0])
def test_sark_exact_for_quadratic_forcing(g):
    """For y' = -lam y + p(t) with p quadratic the final weights reproduce
    the variation-of-constants formula (eq. time_volterra) exactly."""
    import mpmath as mp
    lam = 2.0
    dt = -g / lam
    p = lambda t: 0.3 - 1.1 * t + 0.7 * t * t
    y0, t0 = 0.9, 0.25
    a, b = sark.coefficients(g)
    cs = sark.C_STAGE
    y1 = math.exp(g) * y0 + dt * sum(b[j] * p(t0 + cs[j] * dt) for j in range(4))
    with mp.workdps(40):
        f = lambda th: mp.exp(lam * (th - (t0 + dt))) * (0.3 - 1.1 * th + 0.7 * th * th)
        exact = mp.exp(-lam * dt) * y0 + mp.quad(f, [t0, t0 + dt])
    assert abs(y1 - float(exact)) < 1e-14


def _sark_scalar(lam, mu, dt, T, y0=1.0):
    """Integrate y' = -lam y + mu y with SARK-4 (F = mu y non-stiff)."""
    g = -lam * dt
    a, b = sark.coefficients(g)
    E = [1.0, math.exp(g / 2), math.exp(g / 2), math.exp(g), math.exp(g)]
    y = y0
    for _ in range(int(round(T / dt))):
        F0 = mu * y
        y1 = E[1] * y + dt * a[(1, 0)] * F0
        F1 = mu * y1
        y2 = E[2] * y + dt * (a[(2, 0)] * F0 + a[(2, 1)] * F1)
        F2 = mu * y2
        y3 = E[3] * y + dt * (a[(3, 0)] * F0 + a[(3, 1)] * F1 + a[(3, 2)] * F2)
        F3 = mu * y3
        y = E[4] * y + dt * (b[0] * F0 + b[1] * F1 + b[2] * F2 + b[3] * F3)
    return y


def test_sark_fourth_order():
    """Fourth order on a non-stiff linear coupling (stage coefficients)."""
    lam, mu, T = 3.0, -1.7, 1.0
    exact = math.exp((mu - lam) * T)
    errs = [abs(_sark_scalar(lam, mu, T / n, T) - exact) for n in (8, 16, 32)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.8


def test_sark_stiff_decay_is_exact():
    """With no forcing the update is exactly y_n e^{-lam dt} at any step size."""
    for dt in (1e-3, 0.1, 10.0):
        y = _sark_scalar(100.0, 0.0, dt, dt * 3)
        assert abs(y - math.exp(-300.0 * dt)) < 1e-15


def test_sark_limit_matches_printed_tableau():
    """Golden: table Butcher as printed in the paper."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rk4_tableau.json")))
    a, b = sark.coefficients(-1e-12)
    for k, v in g["a"].items():
        i, j = map(int, k.split(","))
        assert abs(a[(i, j)] - v) < 1e-11
    assert np.allclose(b, g["b"], atol=1e-11)
    assert tuple(sark.C_STAGE) == tuple(g["c"])
