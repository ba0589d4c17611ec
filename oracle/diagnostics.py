"""Flow diagnostics of the ALE solution (oracle).

Test infrastructure only (see ``oracle/__init__``).

Kinetic energy (Section 7.2, the definition after eq. TGV_deformation):
  E_K = 1 / (rho_inf |Omega|) * integral over Omega of rho u.u / 2,
with rho u = c m (Section 2), so the integrand is c^2 |m|^2 / (2 rho).  The
integral is taken element by element with the cubature rule of the relaxation
term (collapsed Gauss-Jacobi, exact to degree 3N) applied to the degree-N
density and momentum of the element, at the current vertex positions.  |Omega|
is the current mesh volume.

Dissipation rate epsilon_1 = -dE_K/dt (Section 7.2).  Here it is the exact time
derivative of the discrete E_K along the semi-discrete ALE system at the
current state: the nodal values of density and momentum change at fixed
reference coordinates by F(q) (the conserved fields carry no stiff part), and
the element Jacobian changes by dJ/dt = J div(w) for the element-wise linear
grid velocity w (Section 5).  Hence, with I = sum_e J_e sum_c w_c e_c,
  dI/dt = sum_e J_e [div(w_e) sum_c w_c e_c
                     + sum_c w_c (de/drho rhodot_c + de/dm . mdot_c)],
  dE_K/dt = (dI/dt - E_K rho_inf d|Omega|/dt) / (rho_inf |Omega|),
with rhodot, mdot the cubature-point values of F.

Wall force (Section 7.3, the drag coefficient c_D = F_D / (rho_inf u_inf^2 c / 2);
Section 7.4 splits the force into pressure and viscous parts).  On every wall
face of the fluid mesh, with n the outward unit normal of the fluid element
(pointing into the body), the force of the fluid on the body is
  F_p = integral of p n ds,       p = rho RT = c^2 rho  (equation of state),
  F_v = -integral of sigma n ds,  sigma the deviatoric stress of Section 2,
       sigma_ab = -c^2 (S_ab - m_a m_b / rho),
S the stress moments (S_xy = q4, S_xx = sqrt2 q5, S_yy = sqrt2 q6 in 2D; the
3D tensor form of the oracle's moment system otherwise).  The face integral
of the nodal values uses the face mass matrix (the integral of each face
node's Lagrange function over the face), scaled by the physical face measure.
"""
from __future__ import annotations

import math

import numpy as np

from . import gbsystem as gb
from .mesh import WALL
from .rhs import element_geometry, rhs

SQ2 = math.sqrt(2.0)


def _cubature_values(mesh, q):
    """Density and momentum at the cubature points, [n, Nc] and [n, dim, Nc]."""
    ref, dim = mesh.ref, mesh.dim
    qc = q @ ref.Icub.T                                  # [n, NF, Nc]
    return qc[:, 0], qc[:, 1:1 + dim]


def grid_divergence(mesh, xv, wv, elems=None):
    """div(w) of the element-wise linear grid velocity, [n]."""
    dim = mesh.dim
    E = np.arange(mesh.K) if elems is None else np.asarray(elems, np.int64)
    _, Ginv, _, _, _ = element_geometry(mesh, xv, E)    # Ginv[n, a, i] = dr_a/dx_i
    W = wv[mesh.etov[E]]                                 # [n, dim+1, dim]
    # dw_i/dr_a for the P1 interpolant on the reference simplex
    dWdr = np.stack([(W[:, a + 1] - W[:, 0]) / 2 for a in range(dim)], axis=-1)   # [n, i, a]
    return np.einsum("nia,nai->n", dWdr, Ginv)


def kinetic_energy(mesh, prm, q, xv, rho_inf=1.0):
    """(E_K, |Omega|) of the state q [K, NF, Np] at vertex positions xv."""
    ref = mesh.ref
    J = element_geometry(mesh, xv, np.arange(mesh.K))[0]
    rho, m = _cubature_values(mesh, q)
    e = 0.5 * prm.c ** 2 * (m * m).sum(axis=1) / rho    # [K, Nc]
    integral = np.einsum("k,c,kc->", J, ref.cub_w, e)
    volume = float(J.sum() * ref.cub_w.sum())
    return integral / (rho_inf * volume), volume


def energy_rate(mesh, prm, q, xv, wv, rho_inf=1.0):
    """dE_K/dt of the semi-discrete system at state q, positions xv and
    vertex grid velocity wv (the dissipation rate is its negative)."""
    ref = mesh.ref
    J = element_geometry(mesh, xv, np.arange(mesh.K))[0]
    divw = grid_divergence(mesh, xv, wv)
    F = rhs(mesh, prm, q, xv, wv)
    rho, m = _cubature_values(mesh, q)
    rdot, mdot = _cubature_values(mesh, F)
    c2 = prm.c ** 2
    e = 0.5 * c2 * (m * m).sum(axis=1) / rho
    de = c2 * (m * mdot).sum(axis=1) / rho - 0.5 * c2 * (m * m).sum(axis=1) * rdot / rho ** 2
    w = ref.cub_w
    integral = np.einsum("k,c,kc->", J, w, e)
    dintegral = np.einsum("k,c,kc->", J * divw, w, e) + np.einsum("k,c,kc->", J, w, de)
    volume = J.sum() * w.sum()
    dvolume = (J * divw).sum() * w.sum()
    EK = integral / (rho_inf * volume)
    return (dintegral - EK * rho_inf * dvolume) / (rho_inf * volume)


def deviatoric_stress(dim, qv, c):
    """sigma [dim, dim, ...] from moments qv [NF, ...] (Section 2)."""
    rho = qv[0]
    m = [qv[1 + d] for d in range(dim)]
    if dim == 2:
        S = [[SQ2 * qv[4], qv[3]], [qv[3], SQ2 * qv[5]]]
    else:
        off = {(0, 1): 4, (0, 2): 5, (1, 2): 6}
        S = [[None] * 3 for _ in range(3)]
        for a in range(3):
            S[a][a] = SQ2 * qv[7 + a]
            for b in range(a + 1, 3):
                S[a][b] = S[b][a] = qv[off[(a, b)]]
    return np.array([[-c * c * (S[a][b] - m[a] * m[b] / rho) for b in range(dim)] for a in range(dim)])


def wall_force(mesh, prm, q, xv):
    """(F_p [dim], F_v [dim]): pressure and viscous force of the fluid on the
    body over all wall faces, at vertex positions xv."""
    ref, dim = mesh.ref, mesh.dim
    Fp = np.zeros(dim)
    Fv = np.zeros(dim)
    ee, ff = np.nonzero(mesh.face_tag == WALL)
    if ee.size == 0:
        return Fp, Fv
    _, _, nrm, meas, _ = element_geometry(mesh, xv, ee)
    Nfp = ref.Nfp
    for f in range(ref.Nfaces):
        sel = ff == f
        if not np.any(sel):
            continue
        # integral of each face node's Lagrange function over the reference face
        wface = ref.Mf[:, f * Nfp:(f + 1) * Nfp].sum(axis=0)           # [Nfp]
        scale = meas[sel, f] / ref.face_area[f]                          # [n]
        qv = q[ee[sel]][:, :, ref.fmask[f]].transpose(1, 0, 2)           # [NF, n, Nfp]
        n = nrm[sel, f]                                                  # [n, dim]
        p = prm.c ** 2 * qv[0]                                           # [n, Nfp]
        sig = deviatoric_stress(dim, qv, prm.c)                          # [dim, dim, n, Nfp]
        for a in range(dim):
            Fp[a] += np.einsum("n,j,nj->", scale, wface, p * n[:, a, None])
            sn = sum(sig[a, b] * n[:, b, None] for b in range(dim))
            Fv[a] -= np.einsum("n,j,nj->", scale, wface, sn)
    return Fp, Fv
