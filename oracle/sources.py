"""Initial boundary densities rho0 projected onto the basis (paper Sec. 4: Eq. RhoNeumann
and Eq. SourceRho are projected onto the finite basis of Eq. FBApprox the same way).

Galerkin projection in the flux measure: the coefficient vector of a density
f(s, d) on slot (j, l) is (I_P kron G^{-1}) [int b_p(s) psi_k(d) f(s, d) ds cos(theta) dOmega].
All sources used here separate, f(s, d) = sigma(s) alpha(d).

Source kinds (all scaled to a total flux int f ds dp = ``flux``):
  face_flux   sigma = const on every boundary face lying in the plane x_axis = value,
              alpha = (3/(2 pi)) cos(theta) (normal-incidence weighted, unit flux per area);
  gauss_patch sigma = exp(-|s-c|^2/(2 s^2))/(2 pi s^2) on the faces of that plane,
              alpha as above;
  points      sigma = delta(s - s0) on the boundary face containing s0, alpha = 1/pi
              (isotropic in p, unit flux);
  face_normal sigma as for face_flux, direction fixed along the inward normal: the
              normal-incidence density of Eq. RhoNeumann (Sec. 4.1), alpha =
              delta(rho)/(2 pi rho) in the polar coordinates rho = sin(theta), phi of
              the tangential momentum (unit flux per area).
"""
from __future__ import annotations

import numpy as np

from . import basis
from .assemble import Basis
from .geometry import barycentric_3d


def project_angular(alpha, D, family, nu=64, nphi=128):
    """G^{-1} int alpha(cos theta, phi) psi_k cos(theta) dOmega by a product Gauss
    rule in (u = cos theta, phi) (exact for the Legendre family)."""
    xu, wu = np.polynomial.legendre.leggauss(nu)
    xp, wp = np.polynomial.legendre.leggauss(nphi)
    u = 0.5 * (xu + 1.0)
    phi = np.pi * (xp + 1.0)
    U, PHI = np.meshgrid(u, phi, indexing="ij")
    W = np.outer(0.5 * wu, np.pi * wp) * U          # u du dphi
    psi = basis.momentum(U.ravel(), PHI.ravel(), D, family)
    rhs = psi.T @ (W.ravel() * alpha(U.ravel(), PHI.ravel()))
    return np.linalg.solve(basis.gram(D, family), rhs)


def project_pole(D, family, nphi=128):
    """G^{-1} int delta(rho)/(2 pi rho) psi_k rho drho dphi: the momentum functions at
    the pole (theta = 0) averaged over phi (Gauss-Legendre in phi, exact for both
    families), then the Gram solve."""
    xp, wp = np.polynomial.legendre.leggauss(nphi)
    phi = np.pi * (xp + 1.0)
    psi = basis.momentum(np.ones_like(phi), phi, D, family)      # cos(theta) = 1
    avg = (0.5 * wp) @ psi
    return np.linalg.solve(basis.gram(D, family), avg)


def _plane_slots(mesh, axis, value):
    out = []
    for j in range(mesh.nt):
        for l in range(4):
            if mesh.nbr[j, l] < 0 and np.all(mesh.verts[mesh.fverts[j, l]][:, axis] == value):
                out.append((j, l))
    return out


def _triangle_rule(n=24):
    """Collapsed (Duffy) Gauss rule on the reference triangle: barycentrics [Q,3], weights (sum 1/2)."""
    x, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    WW = np.outer(wu, wu) * (1.0 - U)
    l1 = U.ravel()
    l2 = (V * (1.0 - U)).ravel()
    lam = np.stack([1.0 - l1 - l2, l1, l2], axis=1)
    return lam, WW.ravel()


def _flux_alpha(u, phi):
    return 1.5 / np.pi * u


def _iso_alpha(u, phi):
    return np.full_like(u, 1.0 / np.pi)


def project(mesh, bs: Basis, src):
    """rho0 [nrhs][4*nt*K] for a source description (see module doc)."""
    P, M, K = bs.P, bs.M, bs.K
    nt = mesh.nt
    kind = src["kind"]
    flux = float(src.get("flux", 1.0))
    if kind == "face_normal":
        ang = project_pole(bs.mom_degree, bs.mom_family)
        slots = _plane_slots(mesh, src["axis"], src["value"])
        total = sum(mesh.area[j, l] for (j, l) in slots)
        rho0 = np.zeros((1, 4 * nt, P, M))
        for (j, l) in slots:
            rho0[0, 4 * j + l, 0, :] = flux / total * np.sqrt(mesh.area[j, l]) * ang
        return rho0.reshape(1, -1)
    if kind in ("face_flux", "gauss_patch"):
        ang = project_angular(_flux_alpha, bs.mom_degree, bs.mom_family)
        slots = _plane_slots(mesh, src["axis"], src["value"])
        rho0 = np.zeros((1, 4 * nt, P, M))
        if kind == "face_flux":
            total = sum(mesh.area[j, l] for (j, l) in slots)
            for (j, l) in slots:
                # int b_0 * const ds = sqrt(area) * const; higher p integrate to 0
                rho0[0, 4 * j + l, 0, :] = flux / total * np.sqrt(mesh.area[j, l]) * ang
        else:
            lam_ref, w_ref = _triangle_rule()
            c = np.asarray(src["center"], dtype=np.float64)
            s2 = float(src["sigma"]) ** 2
            for (j, l) in slots:
                V = mesh.verts[mesh.fverts[j, l]]
                pts = lam_ref @ V
                A = mesh.area[j, l]
                gs = np.exp(-np.sum((pts - c) ** 2, axis=1) / (2 * s2)) / (2 * np.pi * s2)
                b = basis.position_basis(lam_ref, A, bs.pos_order)       # [Q, P]
                mom = b.T @ (w_ref * 2.0 * A * gs)                       # int b_p sigma ds
                rho0[0, 4 * j + l] = flux * np.outer(mom, ang)
        return rho0.reshape(1, -1)
    if kind == "points":
        xyz = np.asarray(src["xyz"], dtype=np.float64)
        ang = project_angular(_iso_alpha, bs.mom_degree, bs.mom_family)
        rho0 = np.zeros((xyz.shape[0], 4 * nt, P, M))
        bslots = [(j, l) for j in range(nt) for l in range(4) if mesh.nbr[j, l] < 0]
        for r, s0 in enumerate(xyz):
            for (j, l) in bslots:
                V = mesh.verts[mesh.fverts[j, l]]
                nrm = np.cross(V[1] - V[0], V[2] - V[0])
                if abs((s0 - V[0]) @ nrm) > 1e-12 * np.linalg.norm(nrm):
                    continue
                lam = barycentric_3d(s0[None, :], V[0], V[1], V[2])[0]
                if np.all(lam >= -1e-12):
                    b = basis.position_basis(lam, mesh.area[j, l], bs.pos_order)
                    rho0[r, 4 * j + l] = flux * np.outer(b, ang)
                    break
            else:
                raise ValueError(f"source point {s0} is not on the mesh boundary")
        return rho0.reshape(xyz.shape[0], -1)
    raise ValueError(f"unknown source kind {kind}")
