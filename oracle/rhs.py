"""Semi-discrete right-hand side F(q) of the ALE nodal DG scheme (oracle).

Test infrastructure only (see ``oracle/__init__``).

Section 3, eq. semi_discrete_form, with the time split of Section 4
(eq. time_split): F(q) collects every term of the semi-discrete form except the
stiff linear relaxation -Lambda q, which the SARK update integrates exactly:

  F = (A + v_G) . D_x q                      volume term (eq. ale_bns)
    + L ( F_num(q* - q-) )                   upwind surface term (eq. upwind_flux)
    + P Ntilde(I q)                          cubature relaxation source

Readings taken where the paper is ambiguous:
  * Upwind sign.  The system is q_t + B . grad q = 0 with B_d = c M_d - w_d I
    (A_d = -c M_d, w the grid velocity).  The physically upwind strong-form
    surface term is B_n^-(q- - q+), B_n^- the non-positive part; the printed
    Lambda+ / Lambda- labels are read with that physical meaning.
  * flux_mode "split" (the paper, eq. upwind_flux): the stationary part and the
    ALE part are upwinded separately, B_n^- = (c M_n)^- + min(-w.n, 0) I.
    flux_mode "relative": the characteristic speeds c lambda_k - w.n are
    upwinded together, B_n^- = (c M_n - (w.n) I)^-.
  * For affine elements J^e P^e equals the reference projection
    P = M^-1 I^T diag(w_c) (eq. semi_discrete_form).
The eigen-decomposition of c M_n uses ``numpy.linalg.eigh`` on the explicit
matrix, once per face (the normal is constant on an affine face).

Boundary faces (parity unpinned against the paper, which names a perfectly
matched layer and walls without giving their form): a wall face takes the
ghost state rho+ = rho-, m+ = 2 rho- w / c - m-, S+ = S- (no slip relative to
the moving wall); a far-field face takes q+ = q_inf.  An optional sponge adds
-sigma(r) (q - q_inf), sigma = sigma_max ((r - r0)/(r1 - r0))^2 for r0 < r < r1,
r the distance of the node from the sponge centre.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import gbsystem as gb
from .mesh import FARFIELD, WALL


@dataclass
class Params:
    c: float = 1.0
    tau: float = 1.0
    flux_mode: str = "split"
    q_inf: np.ndarray | None = None          # [NF] far-field / sponge state
    sponge: tuple | None = None              # (cx, cy, r0, r1, sigma_max)


def element_geometry(mesh, xv: np.ndarray, elems: np.ndarray):
    """Affine map data of the elements at vertex positions xv (Section 3):
    J = det G with G = dx/dr; the inverse metric dr/dx; outward unit normals and
    physical face measures."""
    dim = mesh.dim
    P = xv[mesh.etov[elems]]                                     # [n, dim+1, dim]
    G = np.stack([(P[:, a + 1] - P[:, 0]) / 2 for a in range(dim)], axis=-1)  # [n, i, a]
    J = np.linalg.det(G)
    if np.any(J <= 0):
        raise ValueError("element inverted (J <= 0)")
    Ginv = np.linalg.inv(G)                                      # [n, a, i] = dr_a/dx_i
    normals, meas = [], []
    for fv in mesh.ref.faces:
        opp = [v for v in range(dim + 1) if v not in fv][0]
        A = P[:, fv[0]]
        if dim == 2:
            t = P[:, fv[1]] - A
            n = np.stack([t[:, 1], -t[:, 0]], axis=1)
            m = np.linalg.norm(t, axis=1)
        else:
            n = np.cross(P[:, fv[1]] - A, P[:, fv[2]] - A)
            m = 0.5 * np.linalg.norm(n, axis=1)
        n = n / np.linalg.norm(n, axis=1)[:, None]
        # orient away from the opposite vertex
        s = np.sign(np.einsum("nd,nd->n", n, A - P[:, opp]))
        normals.append(n * s[:, None])
        meas.append(m)
    return J, Ginv, np.stack(normals, axis=1), np.stack(meas, axis=1), P


def rhs(mesh, prm: Params, q: np.ndarray, xv: np.ndarray, wv: np.ndarray, elems=None) -> np.ndarray:
    """F(q) on the elements ``elems`` (default all) for the geometry xv and the
    vertex grid velocity wv.  q is [K, NF, Np] over the whole mesh."""
    ref, dim, K = mesh.ref, mesh.dim, mesh.K
    NF = gb.n_fields(dim)
    E = np.arange(K) if elems is None else np.asarray(elems, np.int64)
    J, Ginv, nrm, meas, P = element_geometry(mesh, xv, E)
    W = wv[mesh.etov[E]]                                         # [n, dim+1, dim]
    wn = np.einsum("pv,kvd->kpd", ref.bary, W)                   # nodal P1 velocity
    xn = np.einsum("pv,kvd->kpd", ref.bary, P)                   # nodal positions
    Md = gb.flux_patterns(dim)
    qe = q[E]                                                    # [n, NF, Np]

    # volume term: chain rule on reference derivatives, then A.grad + w.grad
    dq_dr = [qe @ ref.D[a].T for a in range(dim)]                # D_a applied per field
    grad = [sum(Ginv[:, a, i][:, None, None] * dq_dr[a] for a in range(dim)) for i in range(dim)]
    F = np.zeros_like(qe)
    for i in range(dim):
        F += -prm.c * (Md[i] @ grad[i])
        F += wn[:, None, :, i] * grad[i]

    # surface term
    qflat = q.transpose(0, 2, 1).reshape(K * ref.Np, NF)
    Nfp = ref.Nfp
    for f in range(ref.Nfaces):
        fm = ref.fmask[f]
        qm = qe[:, :, fm]                                        # [n, NF, Nfp]
        qp = qflat[mesh.vmapP[E, f]].transpose(0, 2, 1).copy()   # [n, NF, Nfp]
        n = nrm[:, f]                                            # [n, dim]
        wdn = np.einsum("kpd,kd->kp", wn[:, fm], n)              # [n, Nfp]
        tag = mesh.face_tag[E, f]
        if np.any(tag == WALL):
            sel = tag == WALL
            rho = qm[sel, 0]
            qp[sel] = qm[sel]
            for d in range(dim):
                qp[sel, 1 + d] = 2.0 * rho * wn[sel][:, fm, d] / prm.c - qm[sel, 1 + d]
        if np.any(tag == FARFIELD):
            qp[tag == FARFIELD] = np.asarray(prm.q_inf)[None, :, None]
        Mn = np.einsum("kd,dgf->kgf", n, np.stack(Md))
        lam, R = np.linalg.eigh(prm.c * Mn)                      # [n, NF], [n, NF, NF]
        jump = qm - qp
        if prm.flux_mode == "split":
            Bm = (R * np.minimum(lam, 0.0)[:, None, :]) @ R.transpose(0, 2, 1)
            fl = Bm @ jump + np.minimum(-wdn, 0.0)[:, None, :] * jump
        elif prm.flux_mode == "relative":
            sp = np.minimum(lam[:, :, None] - wdn[:, None, :], 0.0)     # [n, NF(char), Nfp]
            cj = R.transpose(0, 2, 1) @ jump                             # characteristic jumps
            fl = R @ (sp * cj)
        else:
            raise ValueError(prm.flux_mode)
        fscale = meas[:, f] / ref.face_area[f] / J
        fl = fl * fscale[:, None, None]
        F += fl @ ref.LIFT[:, f * Nfp:(f + 1) * Nfp].T

    # relaxation source: interpolate to cubature points, Ntilde, project
    qc = qe @ ref.Icub.T
    nt = gb.ntilde(dim, qc.transpose(1, 0, 2), prm.tau).transpose(1, 0, 2)
    F += nt @ ref.Pcub.T

    if prm.sponge is not None:
        cx, cy, r0, r1, smax = prm.sponge
        r = np.hypot(xn[:, :, 0] - cx, xn[:, :, 1] - cy)
        xi = np.clip((r - r0) / (r1 - r0), 0.0, 1.0)
        sig = smax * xi * xi
        F += -sig[:, None, :] * (qe - np.asarray(prm.q_inf)[None, :, None])
    return F
