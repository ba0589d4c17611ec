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
        # face matching: key = wrapped face centroid + wrapped sorted vertex
        # coordinates (on meshes only two cells per period two different faces
        # can share a wrapped vertex set, never a wrapped centroid)
        scale = max(float(np.ptp(self.vx, axis=0).max()), 1.0)
        nf = ref.Nfaces
        K = self.K
        fverts = np.array(ref.faces)                              # [nf, dim]
        FP = P[:, fverts]                                         # [K, nf, dim(verts), dim]
        cen = _wrap(FP.mean(axis=2), lo, self.period)             # [K, nf, dim]
        vw = _wrap(FP, lo, self.period)
        qv = np.round(vw / scale * 1e8).astype(np.int64)          # [K, nf, nv_f, dim]
        # sort the vertices of each face lexicographically (stable passes,
        # least significant coordinate first)
        keys_v = qv.reshape(K * nf, dim, dim)                     # [face, vertex, coord]
        perm = np.tile(np.arange(dim), (K * nf, 1))
        for d in reversed(range(dim)):
            col = np.take_along_axis(keys_v[:, :, d], perm, axis=1)
            perm = np.take_along_axis(perm, np.argsort(col, axis=1, kind="stable"), axis=1)
        srt = np.take_along_axis(keys_v, perm[:, :, None], axis=1).reshape(K * nf, dim * dim)
        keys = np.concatenate([np.round(cen / scale * 1e8).astype(np.int64).reshape(K * nf, dim), srt], axis=1)
        _, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
        inv = inv.ravel()
        if np.any(counts > 2):
            raise ValueError("more than two faces share a key")
        self.etoe = np.tile(np.arange(K)[:, None], (1, nf))
        self.etof = np.tile(np.arange(nf)[None, :], (K, 1))
        srt_idx = np.argsort(inv, kind="stable")
        grp = inv[srt_idx]
        pair = np.nonzero(grp[1:] == grp[:-1])[0]
        a, b = srt_idx[pair], srt_idx[pair + 1]
        ea, fa, eb, fb = a // nf, a % nf, b // nf, b % nf
        self.etoe[ea, fa], self.etof[ea, fa] = eb, fb
        self.etoe[eb, fb], self.etof[eb, fb] = ea, fa
        matched = np.zeros((K, nf), bool)
        matched[ea, fa] = True
        matched[eb, fb] = True
        self.face_tag = np.zeros((K, nf), np.int8)
        if face_tag is not None:
            self.face_tag[:] = np.asarray(face_tag, np.int8)
        if np.any(~matched & (self.face_tag == INTERIOR)):
            raise ValueError("unmatched face without a boundary tag")
        self.face_tag[matched] = INTERIOR
        # node pairing on matched faces by coordinates modulo the period
        Np, Nfp = ref.Np, ref.Nfp
        self.vmapP = (np.arange(K)[:, None, None] * Np + ref.fmask[None, :, :]).astype(np.int64)
        ee_all, ff_all = np.nonzero(matched)
        for c0 in range(0, ee_all.size, 65536):
            ee, ff = ee_all[c0:c0 + 65536], ff_all[c0:c0 + 65536]
            e2, f2 = self.etoe[ee, ff], self.etof[ee, ff]
            mine = self.nodes_x[ee[:, None], ref.fmask[ff]]              # [M, Nfp, dim]
            other = self.nodes_x[e2[:, None], ref.fmask[f2]]             # [M, Nfp, dim]
            d = _min_image(mine[:, :, None, :] - other[:, None, :, :], self.period)
            dist = np.linalg.norm(d, axis=-1)                            # [M, Nfp, Nfp]
            j = np.argmin(dist, axis=2)
            if np.any(np.take_along_axis(dist, j[..., None], axis=2) > 1e-8 * scale):
                raise ValueError("face nodes do not match")
            self.vmapP[ee, ff] = e2[:, None] * Np + ref.fmask[f2[:, None], j]

    def neighbours(self, elems: np.ndarray) -> np.ndarray:
        """Elements sharing a face with any element of ``elems`` (inclusive)."""
        elems = np.unique(np.asarray(elems, np.int64))
        return np.unique(np.concatenate([elems, self.etoe[elems].ravel()]))
