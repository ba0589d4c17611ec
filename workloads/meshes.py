"""Synthetic simplex meshes shaped like the paper's workloads.

Every generator returns (vx [nv, dim] float64, etov [K, dim+1] int32,
period [dim] float64 (0 = not periodic), face_tag [K, dim+1] int8 or None),
with positively oriented elements.  Periodic meshes keep separate vertices on
opposite sides of the box (no vertex identification) so every element is
geometrically contiguous; the solver pairs faces modulo the period.
Face tags: 0 interior / periodic, 1 wall, 2 far field.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _orient(vx: np.ndarray, etov: np.ndarray) -> np.ndarray:
    """Swap two vertices of every negatively oriented element."""
    P = vx[etov]
    dim = vx.shape[1]
    G = np.stack([P[:, a + 1] - P[:, 0] for a in range(dim)], axis=-1)
    neg = np.linalg.det(G) < 0
    etov = etov.copy()
    etov[neg, 1], etov[neg, 2] = etov[neg, 2].copy(), etov[neg, 1].copy()
    return etov


def periodic_square(n: int, lo: float = -1.0, hi: float = 1.0, seed: int | None = 0,
                    jitter: float = 0.05):
    """[lo,hi]^2 with n x n quads, each split into two triangles.

    With a seed, each quad's diagonal is drawn from numpy.random.default_rng(seed)
    and interior vertices are moved by U(-jitter h, jitter h) per coordinate
    (h = quad size); boundary vertices stay on the box so periodic images
    match.  seed=None gives the regular mesh with all diagonals one way.
    """
    h = (hi - lo) / n
    g = np.linspace(lo, hi, n + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    vx = np.stack([X.ravel(), Y.ravel()], axis=1)
    rng = np.random.default_rng(seed) if seed is not None else None
    diag = rng.integers(0, 2, size=n * n) if rng is not None else np.zeros(n * n, int)
    if rng is not None and jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=vx.shape)
        ij = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy"), -1).reshape(-1, 2)
        interior = (ij[:, 0] > 0) & (ij[:, 0] < n) & (ij[:, 1] > 0) & (ij[:, 1] < n)
        vx[interior] += d[interior]
    vid = lambda i, j: j * (n + 1) + i
    tris = []
    for j in range(n):
        for i in range(n):
            a, b, c, d_ = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if diag[j * n + i] == 0:
                tris += [(a, b, c), (a, c, d_)]
            else:
                tris += [(a, b, d_), (b, c, d_)]
    etov = _orient(vx, np.array(tris, np.int64)).astype(np.int32)
    return vx, etov, np.array([hi - lo, hi - lo]), None


def kuhn_cube(n: int, lo: float = -math.pi, hi: float = math.pi):
    """[lo,hi]^3 with n^3 cubes, each split into the 6 Kuhn (Freudenthal)
    tetrahedra along the main diagonal.  The split is the same in every cube,
    so the mesh is conforming, also across the periodic faces."""
    g = np.linspace(lo, hi, n + 1)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    vx = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)          # cube corners, x fastest
    vid = lambda p: (p[:, 2] * (n + 1) + p[:, 1]) * (n + 1) + p[:, 0]
    unit = np.eye(3, dtype=np.int64)
    per_cube = []
    for perm in itertools.permutations(range(3)):
        p = base.copy()
        vs = [vid(p)]
        for ax in perm:
            p = p + unit[ax]
            vs.append(vid(p))
        per_cube.append(np.stack(vs, axis=1))
    tets = np.stack(per_cube, axis=1).reshape(-1, 4)                     # cube-major order
    etov = _orient(vx, tets.astype(np.int64)).astype(np.int32)
    L = hi - lo
    return vx, etov, np.array([L, L, L]), None


def naca_half_thickness(x: np.ndarray, t: float) -> np.ndarray:
    """NACA 4-digit symmetric half thickness (closed trailing edge)."""
    x = np.clip(x, 0.0, 1.0)
    return 5 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x**2 + 0.2843 * x**3 - 0.1036 * x**4)


def ogrid_airfoil(n_r: int, n_theta: int, radius: float = 20.0, thickness: float = 0.12,
                  first_layer: float = 2e-3):
    """O-grid around a NACA 00xx profile with chord [0,1]: n_theta points around
    the body (cosine clustered at leading and trailing edge) times n_r radial
    layers stretched geometrically out to a circle of the given radius about
    (0.5, 0).  Each quad is split into two triangles.  Body faces are walls,
    outer faces far field; the circumferential seam shares vertices."""
    phi = 2 * math.pi * np.arange(n_theta) / n_theta
    xs = 0.5 * (1 + np.cos(phi))
    ys = np.where(phi <= math.pi, 1.0, -1.0) * naca_half_thickness(xs, thickness)
    ys[0] = 0.0
    inner = np.stack([xs, ys], axis=1)
    outer = np.stack([0.5 + radius * np.cos(phi), radius * np.sin(phi)], axis=1)
    # geometric stretching with the first layer thickness ~ first_layer
    span = radius
    lo_g, hi_g = 1.0 + 1e-9, 2.0
    for _ in range(200):
        gmid = 0.5 * (lo_g + hi_g)
        first = span * (gmid - 1) / (gmid**n_r - 1)
        if first > first_layer:
            lo_g = gmid
        else:
            hi_g = gmid
    g = 0.5 * (lo_g + hi_g)
    s = (g ** np.arange(n_r + 1) - 1) / (g**n_r - 1)
    vx = (inner[None, :, :] + s[:, None, None] * (outer - inner)[None, :, :]).reshape(-1, 2)
    k, j = np.meshgrid(np.arange(n_r, dtype=np.int64), np.arange(n_theta, dtype=np.int64), indexing="ij")
    a, b = k * n_theta + j, k * n_theta + (j + 1) % n_theta
    c, d = (k + 1) * n_theta + (j + 1) % n_theta, (k + 1) * n_theta + j
    # quad (k, j) -> triangles (a, b, c), (a, c, d), quads in (k, j) order
    tris = np.stack([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], axis=2).reshape(-1, 3)
    etov = _orient(vx, tris)
    # face tags: a face on the body (both vertices in layer 0) is a wall, on the
    # outer circle (both in layer n_r) far field
    layer = np.arange(vx.shape[0]) // n_theta
    face_tag = np.zeros((etov.shape[0], 3), np.int8)
    for f, (u, v) in enumerate(((0, 1), (1, 2), (2, 0))):
        lu, lv = layer[etov[:, u]], layer[etov[:, v]]
        face_tag[(lu == 0) & (lv == 0), f] = 1
        face_tag[(lu == n_r) & (lv == n_r), f] = 2
    return vx, etov.astype(np.int32), np.zeros(2), face_tag
