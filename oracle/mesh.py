"""Mesh connectivity for the oracle: element-to-element and node-to-node maps.

Test infrastructure only (see ``oracle/__init__``).

Section 3 of the paper: K straight-sided, positively oriented simplices; each
face node's interior trace q- is paired with the neighbouring element's trace
q+ at the same physical point.  Periodic directions identify points whose
coordinates differ by a whole period.  Faces with no partner are physical
boundaries and carry a tag (0 interior/periodic, 1 wall, 2 far field).
"""
from __future__ import annotations

import numpy as np

from .refelem import ref_element

INTERIOR, WALL, FARFIELD = 0, 1, 2


def _wrap(x: np.ndarray, lo: np.ndarray, period: np.ndarray) -> np.ndarray:
    """Map coordinates of periodic directions into [lo, lo+period)."""
    out = np.array(x, float, copy=True)
    for d in range(out.shape[-1]):
        P = period[d]
        if P > 0:
            y = np.mod(out[..., d] - lo[d], P)
            y = np.where(np.abs(y - P) < 1e-9 * P, 0.0, y)
            out[..., d] = y + lo[d]
    return out


def _min_image(dx: np.ndarray, period: np.ndarray) -> np.ndarray:
    out = np.array(dx, float, copy=True)
    for d in range(out.shape[-1]):
        P = period[d]
        if P > 0:
            out[..., d] -= P * np.round(out[..., d] / P)
    return out


class Mesh:
    """Connectivity of a simplex mesh for polynomial order N.

    Attributes
      vx [nv, dim], etov [K, dim+1]
      nodes_x [K, Np, dim]  node coordinates on the initial mesh
      etoe, etof [K, Nfaces]  neighbour element / face (self for boundaries)
      face_tag [K, Nfaces]
      vmapP [K, Nfaces, Nfp]  flat index e'*Np + j' of the exterior node
    """

    def __init__(self, dim, N, vx, etov, period=None, face_tag=None, cub_degree=None):
        self.dim, self.N = dim, N
        self.vx = np.asarray(vx, float)
        self.etov = np.asarray(etov, np.int64)
        self.K = self.etov.shape[0]
        self.ref = ref_element(dim, N, cub_degree)
        ref = self.ref
        self.period = np.zeros(dim) if period is None else np.asarray(period, float)
        lo = self.vx.min(axis=0)
        # orientation check: J > 0 for every element
        P = self.vx[self.etov]                       # [K, dim+1, dim]
        G = np.stack([(P[:, a + 1] - P[:, 0]) / 2 for a in range(dim)], axis=-1)
        J = np.linalg.det(G)
        if np.any(J <= 0):
            raise ValueError("mesh has non-positively oriented elements")
        self.nodes_x = np.einsum("nv,kvd->knd", ref.bary, P)
        # face matching by wrapped, sorted vertex coordinates
        scale = max(float(np.ptp(self.vx, axis=0).max()), 1.0)
        keys = {}
        nf = ref.Nfaces
        self.etoe = np.tile(np.arange(self.K)[:, None], (1, nf))
        self.etof = np.tile(np.arange(nf)[None, :], (self.K, 1))
        matched = np.zeros((self.K, nf), bool)
        for e in range(self.K):
            for f, fv in enumerate(ref.faces):
                # wrapped centroid plus wrapped vertex set: on meshes only two
                # cells per period two different faces can share a wrapped
                # vertex set, never a wrapped centroid
                cen = _wrap(P[e, list(fv)].mean(axis=0), lo, self.period)
                pts = _wrap(P[e, list(fv)], lo, self.period)
                key = (tuple(np.round(cen / scale * 1e8).astype(np.int64)),
                       tuple(sorted(tuple(np.round(p / scale * 1e8).astype(np.int64)) for p in pts)))
                if key in keys:
                    e2, f2 = keys.pop(key)
                    self.etoe[e, f], self.etof[e, f] = e2, f2
                    self.etoe[e2, f2], self.etof[e2, f2] = e, f
                    matched[e, f] = matched[e2, f2] = True
                else:
                    keys[key] = (e, f)
        self.face_tag = np.zeros((self.K, nf), np.int8)
        if face_tag is not None:
            self.face_tag[:] = np.asarray(face_tag, np.int8)
        unmatched = ~matched
        if np.any(unmatched & (self.face_tag == INTERIOR)):
            raise ValueError("unmatched face without a boundary tag")
        self.face_tag[matched] = INTERIOR
        # node pairing on matched faces by coordinates modulo the period
        Np, Nfp = ref.Np, ref.Nfp
        self.vmapP = np.zeros((self.K, nf, Nfp), np.int64)
        for e in range(self.K):
            for f in range(nf):
                mine = self.nodes_x[e, ref.fmask[f]]                  # [Nfp, dim]
                if not matched[e, f]:
                    self.vmapP[e, f] = e * Np + ref.fmask[f]
                    continue
                e2, f2 = self.etoe[e, f], self.etof[e, f]
                other = self.nodes_x[e2, ref.fmask[f2]]
                d = _min_image(mine[:, None, :] - other[None, :, :], self.period)
                dist = np.linalg.norm(d, axis=-1)
                j = np.argmin(dist, axis=1)
                if np.any(dist[np.arange(Nfp), j] > 1e-8 * scale):
                    raise ValueError("face nodes do not match")
                self.vmapP[e, f] = e2 * Np + ref.fmask[f2][j]

    def neighbours(self, elems: np.ndarray) -> np.ndarray:
        """Elements sharing a face with any element of ``elems`` (inclusive)."""
        elems = np.unique(np.asarray(elems, np.int64))
        return np.unique(np.concatenate([elems, self.etoe[elems].ravel()]))
