"""Reference simplex element for the oracle (triangle and tetrahedron).

Test infrastructure only (see ``oracle/__init__``).

Follows Section 3 (Spatial Discretization) of the paper: a nodal Lagrange basis
of P_N on Warp & Blend nodes, the mass, face-mass and stiffness operators and
the derived differentiation, lift and projection operators
(eq. semi_discrete_form), and a cubature rule with its interpolation operator
used for the nonlinear relaxation term.

Deliberately different route from the GPU library's host setup so that the two
pin each other:
  * polynomial basis: products of Legendre polynomials P_i(r)P_j(s)(P_k(t)),
    i+j(+k) <= N (not the orthonormal simplex basis);
  * mass / face-mass matrices: assembled by quadrature from their integral
    definitions, faces measured in true reference arc length / area;
  * Gauss rules: ``scipy.special.roots_jacobi`` / numpy Legendre roots.

Reference triangle: (-1,-1), (1,-1), (-1,1).  Reference tetrahedron:
(-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).
Faces are listed as vertex tuples: triangle (0,1), (1,2), (2,0); tetrahedron
(0,1,2), (0,1,3), (1,2,3), (0,2,3).
"""
from __future__ import annotations

import functools
import math

import numpy as np
from numpy.polynomial import legendre as npleg
import mpmath as mp
from scipy.special import roots_jacobi

TRI_VERTS = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
TET_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
TRI_FACES = ((0, 1), (1, 2), (2, 0))
TET_FACES = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))

# Warp & Blend blending parameters alpha (Warburton 2006, optimised for the
# Lebesgue constant), indexed by N-1; values beyond the table use the
# asymptotic choice of that paper.
_ALPHA_TRI = (0.0000, 0.0000, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
              1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258)
_ALPHA_TET = (0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603,
              1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655)


def n_nodes(dim: int, N: int) -> int:
    if dim == 2:
        return (N + 1) * (N + 2) // 2
    return (N + 1) * (N + 2) * (N + 3) // 6


# ----------------------------------------------------------------------------
# 1D Gauss rules
# ----------------------------------------------------------------------------

def lgl_nodes(N: int) -> np.ndarray:
    """Legendre-Gauss-Lobatto nodes on [-1,1]: +-1 and the roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(np.real(npleg.Legendre.basis(N).deriv().roots()))
    return np.concatenate([[-1.0], inner, [1.0]])


def gauss_jacobi(n: int, alpha: float, beta: float):
    """n-point Gauss rule for the weight (1-x)^alpha (1+x)^beta on [-1,1]."""
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, float), np.asarray(w, float)


# ----------------------------------------------------------------------------
# Warp & Blend nodes (Warburton 2006), restated
# ----------------------------------------------------------------------------

def _warp_over_bubble(N: int, r: np.ndarray) -> np.ndarray:
    """(LGL - equispaced) displacement interpolated on the equispaced nodes,
    divided by the bubble (1 - r^2).

    The interpolant vanishes at r = +-1, so the quotient is a polynomial; it is
    evaluated as a sum of Lagrange products with the two end-node factors
    (whose product is r^2 - 1) left out.
    """
    r = np.asarray(r, float)
    req = np.linspace(-1.0, 1.0, N + 1)
    disp = lgl_nodes(N) - req
    out = np.zeros_like(r)
    for i in range(1, N):          # end nodes carry zero displacement
        term = np.full_like(r, disp[i])
        for j in range(N + 1):
            if j == i:
                continue
            term = term / (req[i] - req[j])
            if j != 0 and j != N:
                term = term * (r - req[j])
        # the left-out factors (r - req[0])(r - req[N]) = (r+1)(r-1) = -(1-r^2)
        out += -term
    return out


def _tri_equilateral_shift(N: int, alpha: float, L1, L2, L3):
    """Warp & blend displacement in the equilateral triangle whose barycentric
    coordinates are (L1, L2, L3) (L1 at the top vertex)."""
    b1, b2, b3 = 4 * L2 * L3, 4 * L1 * L3, 4 * L1 * L2
    w1 = b1 * _warp_over_bubble(N, L3 - L2) * (1 + (alpha * L1) ** 2)
    w2 = b2 * _warp_over_bubble(N, L1 - L3) * (1 + (alpha * L2) ** 2)
    w3 = b3 * _warp_over_bubble(N, L2 - L1) * (1 + (alpha * L3) ** 2)
    c2, s2 = math.cos(2 * math.pi / 3), math.sin(2 * math.pi / 3)
    c4, s4 = math.cos(4 * math.pi / 3), math.sin(4 * math.pi / 3)
    dx = w1 + c2 * w2 + c4 * w3
    dy = s2 * w2 + s4 * w3
    return dx, dy


@functools.lru_cache(maxsize=None)
def nodes_tri(N: int) -> np.ndarray:
    """Warp & Blend nodes on the reference triangle, lattice order (rows of
    increasing s outer, increasing r inner).  Returns [Np, 2]."""
    alpha = _ALPHA_TRI[N - 1] if N <= len(_ALPHA_TRI) else 5.0 / 3.0
    L1, L3 = [], []
    for n in range(N + 1):
        for m in range(N + 1 - n):
            L1.append(n / N)
            L3.append(m / N)
    L1 = np.array(L1)
    L3 = np.array(L3)
    L2 = 1.0 - L1 - L3
    x = -L2 + L3
    y = (-L2 - L3 + 2 * L1) / math.sqrt(3.0)
    dx, dy = _tri_equilateral_shift(N, alpha, L1, L2, L3)
    x = x + dx
    y = y + dy
    # equilateral -> reference right triangle via barycentric coordinates
    B1 = (math.sqrt(3.0) * y + 1.0) / 3.0
    B2 = (-3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    B3 = (3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    r = -B2 + B3 - B1
    s = -B2 - B3 + B1
    return np.stack([r, s], axis=1)


@functools.lru_cache(maxsize=None)
def nodes_tet(N: int) -> np.ndarray:
    """Warp & Blend nodes on the reference tetrahedron, lattice order (t outer,
    s middle, r inner).  Returns [Np, 3]."""
    alpha = _ALPHA_TET[N - 1] if N <= len(_ALPHA_TET) else 1.0
    tol = 1e-10
    pts = []
    for n in range(N + 1):
        for m in range(N + 1 - n):
            for q in range(N + 1 - n - m):
                pts.append((-1 + 2 * q / N, -1 + 2 * m / N, -1 + 2 * n / N))
    pts = np.array(pts)
    r, s, t = pts[:, 0], pts[:, 1], pts[:, 2]
    L1 = (1 + t) / 2
    L2 = (1 + s) / 2
    L3 = -(1 + r + s + t) / 2
    L4 = (1 + r) / 2
    v1 = np.array([-1.0, -1 / math.sqrt(3), -1 / math.sqrt(6)])
    v2 = np.array([1.0, -1 / math.sqrt(3), -1 / math.sqrt(6)])
    v3 = np.array([0.0, 2 / math.sqrt(3), -1 / math.sqrt(6)])
    v4 = np.array([0.0, 0.0, 3 / math.sqrt(6)])
    t1 = [v2 - v1, v2 - v1, v3 - v2, v3 - v1]
    t2 = [v3 - 0.5 * (v1 + v2), v4 - 0.5 * (v1 + v2), v4 - 0.5 * (v2 + v3), v4 - 0.5 * (v1 + v3)]
    t1 = [a / np.linalg.norm(a) for a in t1]
    t2 = [a / np.linalg.norm(a) for a in t2]
    X = np.outer(L3, v1) + np.outer(L4, v2) + np.outer(L2, v3) + np.outer(L1, v4)
    shift = np.zeros_like(X)
    for face in range(4):
        if face == 0:
            La, Lb, Lc, Ld = L1, L2, L3, L4
        elif face == 1:
            La, Lb, Lc, Ld = L2, L1, L3, L4
        elif face == 2:
            La, Lb, Lc, Ld = L3, L1, L4, L2
        else:
            La, Lb, Lc, Ld = L4, L1, L3, L2
        w1, w2 = _tri_equilateral_shift(N, alpha, Lb, Lc, Ld)
        blend = Lb * Lc * Ld
        denom = (Lb + 0.5 * La) * (Lc + 0.5 * La) * (Ld + 0.5 * La)
        ok = denom > tol
        blend = np.where(ok, (1 + (alpha * La) ** 2) * blend / np.where(ok, denom, 1.0), blend)
        shift += np.outer(blend * w1, t1[face]) + np.outer(blend * w2, t2[face])
        on_face = (La < tol) & (((Lb > tol).astype(int) + (Lc > tol).astype(int) + (Ld > tol).astype(int)) < 3)
        shift[on_face] = np.outer(w1[on_face], t1[face]) + np.outer(w2[on_face], t2[face])
    X = X + shift
    # equilateral -> reference right tetrahedron
    rhs = X - 0.5 * (v2 + v3 + v4 - v1)
    A = np.stack([0.5 * (v2 - v1), 0.5 * (v3 - v1), 0.5 * (v4 - v1)], axis=1)
    rst = np.linalg.solve(A, rhs.T).T
    return rst


def nodes(dim: int, N: int) -> np.ndarray:
    return nodes_tri(N) if dim == 2 else nodes_tet(N)


def barycentric(dim: int, rs: np.ndarray) -> np.ndarray:
    """Barycentric coordinates w.r.t. the reference vertices, [n, dim+1]."""
    rs = np.atleast_2d(rs)
    if dim == 2:
        r, s = rs[:, 0], rs[:, 1]
        return np.stack([-(r + s) / 2, (1 + r) / 2, (1 + s) / 2], axis=1)
    r, s, t = rs[:, 0], rs[:, 1], rs[:, 2]
    return np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], axis=1)


# ----------------------------------------------------------------------------
# Polynomial basis: products of Legendre polynomials
# ----------------------------------------------------------------------------

def _exponents(dim: int, N: int):
    if dim == 2:
        return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]
    return [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i) for k in range(N + 1 - i - j)]


def _leg_mp(n: int, x):
    """(P_n(x), P_n'(x)) by the three-term recurrence, in mpmath."""
    p0, p1 = mp.mpf(1), x
    d0, d1 = mp.mpf(0), mp.mpf(1)
    if n == 0:
        return p0, d0
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
        d0, d1 = d1, d0 + (2 * k + 1) * p0
    return p1, d1


def basis_mp(dim: int, N: int, pts, deriv=None):
    """Values (or the partial derivative along axis ``deriv``) of the Legendre
    product basis at pts [n, dim], as an mpmath matrix [n, Np].  The points are
    taken exactly from their float64 values."""
    pts = np.atleast_2d(np.asarray(pts, float))
    ex = _exponents(dim, N)
    out = mp.matrix(pts.shape[0], len(ex))
    for p in range(pts.shape[0]):
        xs = [mp.mpf(float(v)) for v in pts[p]]
        tab = [[_leg_mp(n, xs[ax]) for n in range(N + 1)] for ax in range(dim)]
        for k, e in enumerate(ex):
            v = mp.mpf(1)
            for ax in range(dim):
                v *= tab[ax][e[ax]][1 if deriv == ax else 0]
            out[p, k] = v
    return out


def _to_np(m) -> np.ndarray:
    return np.array([[float(m[i, j]) for j in range(m.cols)] for i in range(m.rows)])


# ----------------------------------------------------------------------------
# Cubature: collapsed-coordinate Gauss-Jacobi product rules
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def cubature(dim: int, degree: int):
    """Collapsed Gauss-Jacobi (Stroud) rule exact for total degree <= degree.

    Triangle: r = (1+a)(1-b)/2 - 1, s = b, dr ds = (1-b)/2 da db; Gauss-Legendre
    in a, Gauss-Jacobi(1,0) in b.  Tetrahedron: r = (1+a)(1-b)(1-c)/4 - 1,
    s = (1+b)(1-c)/2 - 1, t = c, Jacobian (1-b)(1-c)^2/8; weights (0,0), (1,0),
    (2,0).  n = ceil((degree+1)/2) points per direction.
    Returns (points [Nc, dim], weights [Nc]).
    """
    n = (degree + 2) // 2
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    if dim == 2:
        A, B = np.meshgrid(a, b, indexing="ij")
        WA, WB = np.meshgrid(wa, wb, indexing="ij")
        r = (1 + A) * (1 - B) / 2 - 1
        s = B
        w = WA * WB / 2
        return np.stack([r.ravel(), s.ravel()], axis=1), w.ravel()
    c, wc = gauss_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    s = (1 + B) * (1 - C) / 2 - 1
    t = C
    w = WA * WB * WC / 8
    return np.stack([r.ravel(), s.ravel(), t.ravel()], axis=1), w.ravel()


# ----------------------------------------------------------------------------
# Reference operators
# ----------------------------------------------------------------------------

class RefElement:
    """Reference operators of eq. semi_discrete_form on the reference simplex.

    Attributes
      r          nodes [Np, dim]
      D          list of dim differentiation matrices D_r, D_s(, D_t) [Np, Np]
      M          reference mass matrix (integral of phi_i phi_j)
      faces      vertex tuples of the reference faces
      fmask      [Nfaces][Nfp] node indices on each face
      face_area  reference measure (length / area) of each face
      LIFT       M^-1 * face mass, [Np, Nfaces*Nfp]; face mass in reference
                 arc length / area (so the physical lift carries the factor
                 (physical face measure / reference face measure) / J)
      cub_r, cub_w   cubature points and weights
      Icub       interpolation nodes -> cubature points [Nc, Np]
      Pcub       projection M^-1 Icub^T diag(w) [Np, Nc]
      bary       barycentric coordinates of the nodes [Np, dim+1] (the P1
                 interpolation table for vertex data)
    """

    def __init__(self, dim: int, N: int, cub_degree: int | None = None):
        self.dim, self.N = dim, N
        self.Np = n_nodes(dim, N)
        self.r = nodes(dim, N)
        self.verts = TRI_VERTS if dim == 2 else TET_VERTS
        self.faces = TRI_FACES if dim == 2 else TET_FACES
        self.Nfaces = dim + 1
        self.Nfp = N + 1 if dim == 2 else (N + 1) * (N + 2) // 2
        # Lagrange basis phi_j = sum_k Vinv[k, j] psi_k, formed in 40-digit
        # arithmetic so the operators are exact to double rounding however
        # ill-conditioned the product basis is at the nodes
        with mp.workdps(40):
            Vinv = basis_mp(dim, N, self.r) ** -1
            # derivative of the unique degree-N interpolant at the nodes
            self.D = [_to_np(basis_mp(dim, N, self.r, deriv=ax) * Vinv) for ax in range(dim)]
            self._Vinv = Vinv

            def lagrange_at(pts):
                return _to_np(basis_mp(dim, N, pts) * Vinv)
        self.lagrange_at = lagrange_at
        # mass matrix from its integral definition (degree 2N integrand)
        qr, qw = cubature(dim, 2 * N)
        Phi = lagrange_at(qr)
        self.M = Phi.T @ (qw[:, None] * Phi)
        self.bary = barycentric(dim, self.r)
        # face node sets: nodes whose barycentric coordinate of the opposite
        # vertex vanishes, ordered by node index
        self.fmask = []
        for fv in self.faces:
            opp = [v for v in range(dim + 1) if v not in fv][0]
            self.fmask.append(np.nonzero(np.abs(self.bary[:, opp]) < 1e-10)[0])
        self.fmask = np.array(self.fmask)
        assert self.fmask.shape == (self.Nfaces, self.Nfp)
        # face mass matrices by quadrature on each reference face
        self.face_area = np.zeros(self.Nfaces)
        Mf = np.zeros((self.Np, self.Nfaces * self.Nfp))
        for f, fv in enumerate(self.faces):
            P = self.verts[list(fv)]
            if dim == 2:
                g, gw = gauss_jacobi(N + 1, 0.0, 0.0)
                lam = np.stack([(1 - g) / 2, (1 + g) / 2], axis=1)
                meas = np.linalg.norm(P[1] - P[0])
                jac = meas / 2.0
            else:
                g, gw = cubature(2, 2 * N)
                lam = barycentric(2, g)
                meas = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
                jac = meas / 2.0
            self.face_area[f] = meas
            xq = lam @ P
            Phif = lagrange_at(xq)
            blk = Phif.T @ ((gw * jac)[:, None] * Phif[:, self.fmask[f]])
            Mf[:, f * self.Nfp:(f + 1) * self.Nfp] = blk
        self.Mf = Mf
        self.LIFT = np.linalg.solve(self.M, Mf)
        # cubature for the relaxation term
        self.cub_degree = 3 * N if cub_degree is None else cub_degree
        self.cub_r, self.cub_w = cubature(dim, self.cub_degree)
        self.Nc = self.cub_w.size
        self.Icub = lagrange_at(self.cub_r)
        self.Pcub = np.linalg.solve(self.M, self.Icub.T * self.cub_w[None, :])


@functools.lru_cache(maxsize=None)
def ref_element(dim: int, N: int, cub_degree: int | None = None) -> RefElement:
    return RefElement(dim, N, cub_degree)
