"""Pins for the oracle's reference element against closed forms.

Monomial integrals over the reference simplex and its faces are evaluated in
exact rational arithmetic (Dirichlet integrals over the unit simplex), so they
are independent of every quadrature the oracle uses.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import refelem as R


def _binom_expand(a):
    """(2u - 1)^a as {power: coefficient}."""
    return {i: Fraction(math.comb(a, i) * 2**i * (-1) ** (a - i)) for i in range(a + 1)}


def simplex_monomial_integral(exps):
    """Exact integral of prod x_d^{e_d} over the reference simplex
    (vertices -1 and the unit corners): x_d = 2 u_d - 1, dx = 2^dim du,
    integral of prod u^i over the unit simplex = prod i! / (sum i + dim)!."""
    dim = len(exps)
    total = Fraction(0)
    expansions = [_binom_expand(e) for e in exps]
    for pw in itertools.product(*[list(ex.items()) for ex in expansions]):
        coef = Fraction(1)
        num = 1
        for (i, cf) in pw:
            coef *= cf
            num *= math.factorial(i)
        s = sum(i for i, _ in pw)
        total += coef * Fraction(num, math.factorial(s + dim))
    return total * 2**dim


def monomials(dim, deg):
    if dim == 2:
        return [(a, b) for a in range(deg + 1) for b in range(deg + 1 - a)]
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a) for c in range(deg + 1 - a - b)]


def evalmono(pts, e):
    v = np.ones(pts.shape[0])
    for d, k in enumerate(e):
        v = v * pts[:, d] ** k
    return v


CASES = [(2, N) for N in range(1, 7)] + [(3, N) for N in range(1, 5)]


@pytest.mark.parametrize("dim,N", CASES)
def test_node_count_and_vertices(dim, N):
    r = R.nodes(dim, N)
    assert r.shape == (R.n_nodes(dim, N), dim)
    verts = R.TRI_VERTS if dim == 2 else R.TET_VERTS
    for v in verts:
        assert np.min(np.linalg.norm(r - v, axis=1)) < 1e-14


@pytest.mark.parametrize("dim,N", CASES)
def test_edge_nodes_are_lgl(dim, N):
    """Warp & Blend places the nodes of every edge at the 1D Gauss-Lobatto
    points (the construction's defining property)."""
    r = R.nodes(dim, N)
    verts = R.TRI_VERTS if dim == 2 else R.TET_VERTS
    lgl = np.sort(R.lgl_nodes(N))
    for a, b in itertools.combinations(range(dim + 1), 2):
        A, B = verts[a], verts[b]
        t = B - A
        # nodes on the segment AB
        lam = (r - A) @ t / (t @ t)
        off = np.linalg.norm(r - A - np.outer(lam, t), axis=1)
        on = (off < 1e-12) & (lam > -1e-12) & (lam < 1 + 1e-12)
        assert on.sum() == N + 1
        assert np.allclose(np.sort(2 * lam[on] - 1), lgl, atol=1e-13)


@pytest.mark.parametrize("dim,N", CASES)
def test_nodes_invariant_under_symmetries(dim, N):
    """The node set is invariant under every vertex permutation of the simplex."""
    r = R.nodes(dim, N)
    B = R.barycentric(dim, r)
    for perm in itertools.permutations(range(dim + 1)):
        Bp = B[:, perm]
        d = np.linalg.norm(Bp[:, None, :] - B[None, :, :], axis=-1)
        assert np.all(d.min(axis=1) < 1e-12)


def test_low_order_nodes_closed_form():
    """N=1: the vertices; N=2: vertices and edge midpoints; N=3 triangle: the
    centroid is the one interior node."""
    assert np.allclose(R.nodes_tri(1), R.TRI_VERTS, atol=1e-15)
    r2 = R.nodes_tri(2)
    mids = [(R.TRI_VERTS[a] + R.TRI_VERTS[b]) / 2 for a, b in ((0, 1), (1, 2), (0, 2))]
    for m in mids:
        assert np.min(np.linalg.norm(r2 - m, axis=1)) < 1e-15
    r3 = R.nodes_tri(3)
    assert np.allclose(r3[5], [-1 / 3, -1 / 3], atol=1e-15)


@pytest.mark.parametrize("dim,N", CASES)
def test_differentiation_exact_on_monomials(dim, N):
    re = R.ref_element(dim, N)
    for e in monomials(dim, N):
        f = evalmono(re.r, e)
        for ax in range(dim):
            if e[ax] == 0:
                d = np.zeros_like(f)
            else:
                e2 = list(e)
                e2[ax] -= 1
                d = e[ax] * evalmono(re.r, e2)
            assert np.abs(re.D[ax] @ f - d).max() < 1e-12 * max(1.0, np.abs(d).max())


@pytest.mark.parametrize("dim,N", CASES)
def test_mass_matrix_matches_exact_integrals(dim, N):
    re = R.ref_element(dim, N)
    mons = monomials(dim, N)
    for e1 in mons:
        for e2 in mons:
            exact = float(simplex_monomial_integral(tuple(a + b for a, b in zip(e1, e2))))
            got = evalmono(re.r, e1) @ re.M @ evalmono(re.r, e2)
            assert abs(got - exact) < 1e-13 * max(1.0, abs(exact))


@pytest.mark.parametrize("dim,N", CASES)
def test_cubature_exact_to_3N(dim, N):
    pts, w = R.cubature(dim, 3 * N)
    assert abs(w.sum() - (2.0 if dim == 2 else 4.0 / 3.0)) < 1e-14
    for e in monomials(dim, 3 * N):
        exact = float(simplex_monomial_integral(e))
        assert abs(w @ evalmono(pts, e) - exact) < 1e-13


@pytest.mark.parametrize("dim,N", CASES)
def test_projection_inverts_interpolation(dim, N):
    re = R.ref_element(dim, N)
    assert np.abs(re.Pcub @ re.Icub - np.eye(re.Np)).max() < 1e-12


def _face_integral_tri(face, e):
    """Exact integral over a reference triangle edge (arc length) of r^a s^b."""
    a, b = e
    if face == 0:      # s = -1, r in [-1,1]
        return (-1) ** b * Fraction(1 - (-1) ** (a + 1), a + 1), 1.0
    if face == 2:      # r = -1, s in [-1,1]
        return (-1) ** a * Fraction(1 - (-1) ** (b + 1), b + 1), 1.0
    # r + s = 0 from (1,-1) to (-1,1): r = 1 - 2l, s = 2l - 1, ds = 2 sqrt2 dl
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            tot += (Fraction(math.comb(a, i)) * (-2) ** i
                    * Fraction(math.comb(b, j)) * 2**j * (-1) ** (b - j) * Fraction(1, i + j + 1))
    return 2 * tot, math.sqrt(2.0)


@pytest.mark.parametrize("N", range(1, 7))
def test_lift_reproduces_face_integrals_tri(N):
    """M LIFT restricted to face f, applied to face-node values of q and
    contracted with nodal values of p, equals the edge integral of p q."""
    re = R.ref_element(2, N)
    ML = re.M @ re.LIFT
    mons = monomials(2, N)
    for f in range(3):
        blk = ML[:, f * re.Nfp:(f + 1) * re.Nfp]
        for e1 in mons:
            for e2 in mons:
                ex, scale = _face_integral_tri(f, tuple(a + b for a, b in zip(e1, e2)))
                got = evalmono(re.r, e1) @ blk @ evalmono(re.r[re.fmask[f]], e2)
                assert abs(got - float(ex) * scale) < 1e-12


@pytest.mark.parametrize("N", range(1, 4))
def test_lift_face_integrals_tet(N):
    """Same for the tetrahedron: every face integral of a product of two
    degree-N polynomials, with the exact value from the face parametrisation
    (a Dirichlet integral times the face-area ratio)."""
    re = R.ref_element(3, N)
    ML = re.M @ re.LIFT
    mons = monomials(3, N)
    for f, fv in enumerate(R.TET_FACES):
        P = R.TET_VERTS[list(fv)]
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        blk = ML[:, f * re.Nfp:(f + 1) * re.Nfp]
        rng = np.random.default_rng(f)
        for _ in range(6):
            e1 = mons[rng.integers(len(mons))]
            e2 = mons[rng.integers(len(mons))]
            # integrand on the face as a polynomial in barycentric (l1, l2) with
            # x = P0 + l1 (P1-P0) + l2 (P2-P0): integrate exactly by expanding
            # with sympy-free rational arithmetic over the unit triangle
            ex = _tet_face_exact(P, tuple(a + b for a, b in zip(e1, e2))) * (area / 0.5)
            got = evalmono(re.r, e1) @ blk @ evalmono(re.r[re.fmask[f]], e2)
            assert abs(got - ex) < 1e-12


def _tet_face_exact(P, e):
    """Integral over the unit triangle (area 1/2) in (l1, l2) of
    prod_d x_d(l)^{e_d}, x = P0 + l1 (P1-P0) + l2 (P2-P0), exact."""
    from collections import defaultdict
    poly = {(0, 0): Fraction(1)}
    for d in range(3):
        lin = {(0, 0): Fraction(int(P[0][d])), (1, 0): Fraction(int(P[1][d] - P[0][d])),
               (0, 1): Fraction(int(P[2][d] - P[0][d]))}
        for _ in range(e[d]):
            new = defaultdict(Fraction)
            for (i, j), a in poly.items():
                for (k, l), b in lin.items():
                    new[(i + k, j + l)] += a * b
            poly = dict(new)
    tot = Fraction(0)
    for (i, j), a in poly.items():
        tot += a * Fraction(math.factorial(i) * math.factorial(j), math.factorial(i + j + 2))
    return float(tot)
