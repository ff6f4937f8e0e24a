"""Receiver energy and its gradients (the adjoint of the stationary solve).

Receiver energy.  The energy carried inside tet j by the boundary density is
the interior density of Eq. IntDens (Sec. 4.1) integrated over the tet.  With
r = r_s + t d, dr = t^2 dt dOmega, the factor cos/|r - r_s|^2 cancels and
    E_j = sum_l int_{face l} int rho(s, d) (1 - exp(-mu_j L(s, d))) / mu_j  ds dp,
L the full chord from s along d (the mu -> 0 limit is L).  J = sum of E_j over
the tets whose centroid lies in a box; J = g . rho for the coefficient vector.

Gradients.  rho solves (I - B(mu)) rho = rho0(w), rho0 = sum_s w_s rho0_s;
lambda solves (I - B)^T lambda = g; then
    dJ/dmu_e = lambda^T (dB/dmu_e) rho + (dg/dmu_e) . rho,   dJ/dw_s = lambda . rho0_s.
Only the blocks of tet e depend on mu_e, through a = mu_e L_max in the spatial
integral: dS/dmu = L_max dS/da with d/da I_{i,m}(a) = -I_{i+1,m}(a).

Everything is evaluated on the same quadrature directions as the blocks of B.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, quadrature
from .assemble import Basis, block_T, in_faces
from .geometry import block_geometry, moment_I
from .mesh import destination


def moment_H(i, m, a):
    """H_{i,m}(a) = int_0^1 u^i (1-u)^m (1 - exp(-a u))/a du (a -> 0: B(i+2, m+1)).

    (B(i+1,m+1) - I_{i,m}(a)) / a for a >= 1e-2; below, the Taylor series
    sum_r (-a)^r / (r+1)! B(i+r+2, m+1)."""
    a = np.asarray(a, dtype=np.float64)
    beta = lambda x, y: math.factorial(x - 1) * math.factorial(y - 1) / math.factorial(x + y - 1)  # noqa: E731
    big = a >= 1e-2
    ab = np.where(big, a, 1.0)
    closed = (beta(i + 1, m + 1) - moment_I(i, m, ab)) / ab
    series = np.zeros_like(a)
    for r in range(12):
        series = series + (-a) ** r / math.factorial(r + 1) * beta(i + r + 2, m + 1)
    return np.where(big, closed, series)


def moment_dH(i, m, a):
    """d/da H_{i,m}(a) = -(H_{i,m}(a) - I_{i+1,m}(a)) / a ... by its series for a < 1e-2."""
    a = np.asarray(a, dtype=np.float64)
    beta = lambda x, y: math.factorial(x - 1) * math.factorial(y - 1) / math.factorial(x + y - 1)  # noqa: E731
    big = a >= 1e-2
    ab = np.where(big, a, 1.0)
    # H = (B - I)/a  =>  H' = (-I' a - (B - I))/a^2 = (a I_{i+1,m} - (B - I_{i,m}))/a^2
    closed = (ab * moment_I(i + 1, m, ab) - (beta(i + 1, m + 1) - moment_I(i, m, ab))) / (ab * ab)
    series = np.zeros_like(a)
    for r in range(1, 13):
        series = series + r * (-1) ** r * a ** (r - 1) / math.factorial(r + 1) * beta(i + r + 2, m + 1)
    return np.where(big, closed, series)


def _corner_moments(moment, area, a):
    """G[q, al, be] = int_T b_al b_be f(a b_O) dA for corners (O, Y, Z) of T with
    f's moments given by `moment(i, m, a)` (I for exp(-a b_O), H for (1-exp)/a)."""
    Q = a.shape[0]
    G = np.zeros((Q, 3, 3))
    for al in range(3):
        for be in range(3):
            e = [0, 0, 0]
            e[al] += 1
            e[be] += 1
            i, jj, kk = e
            G[:, al, be] = 2.0 * area * math.factorial(jj) * math.factorial(kk) \
                / math.factorial(jj + kk + 1) * moment(i, jj + kk + 1, a)
    return G


def _corner_first_moments(moment, area, a):
    """F[q, be] = int_T b_be f(a b_O) dA."""
    Q = a.shape[0]
    F = np.zeros((Q, 3))
    for be in range(3):
        e = [0, 0, 0]
        e[be] += 1
        i, jj, kk = e
        F[:, be] = 2.0 * area * math.factorial(jj) * math.factorial(kk) / math.factorial(jj + kk + 1) \
            * moment(i, jj + kk + 1, a)
    return F


def _inbound_corner_basis(mesh, j, l_in, x, O, pos_order):
    A_in = mesh.area[j, l_in]
    Q = O.shape[0]
    y, z = (x + 1) % 3, (x + 2) % 3
    lam = np.zeros((Q, 3, 3))
    lam[:, 0, :] = O
    lam[:, 1, y] = 1.0
    lam[:, 2, z] = 1.0
    return basis.position_basis(lam, A_in, pos_order)          # [Q, corner, p]


def energy_weights(mesh, j, l_in, l_out, d, mu, pos_order, derivative=False):
    """E[q, p] = int over the start set of face l_out of b_p(s) ell(s) ds with
    ell = (1 - exp(-mu L))/mu (or d ell / d mu when derivative)."""
    O, area, Lmax, x = block_geometry(mesh, j, l_in, l_out, d)
    a = np.where(area > 0.0, mu * Lmax, 0.0)
    L = np.where(area > 0.0, Lmax, 0.0)
    b_in = _inbound_corner_basis(mesh, j, l_in, x, O, pos_order)
    if derivative:
        F = _corner_first_moments(moment_dH, area, a) * (L * L)[:, None]
    else:
        F = _corner_first_moments(moment_H, area, a) * L[:, None]
    return np.einsum("qb,qbp->qp", F, b_in)


def in_box(mesh, box):
    c = mesh.verts[mesh.tets].mean(axis=1)
    lo = np.array(box[0::2])
    hi = np.array(box[1::2])
    return np.all((c >= lo) & (c <= hi), axis=1)


def receiver_functional(mesh, bs: Basis, mu, box, derivative=False):
    """g [4*nt*K] with J = g . rho (or dg/dmu_j in the slots of tet j)."""
    P, M, K = bs.P, bs.M, bs.K
    g = np.zeros((mesh.nt, 4, P, M))
    for j in np.nonzero(in_box(mesh, box))[0]:
        for l_in in range(4):
            for l_out in in_faces(l_in):
                d, W = quadrature.block_nodes(mesh, j, l_in, l_out, bs.quad_n, bs.rule)
                E = energy_weights(mesh, j, l_in, l_out, d, mu[j], bs.pos_order, derivative)
                ci, pi_ = basis.direction_angles(d, mesh.frame[j, l_in])
                psi = basis.momentum(ci, pi_, bs.mom_degree, bs.mom_family)
                g[j, l_in] += np.einsum("q,qp,qk->pk", W, E, psi)
    return g.reshape(-1)


def dS_dmu(mesh, j, l_in, l_out, d, mu, pos_order):
    """dS/dmu[q, p', p] for the spatial integral of geometry.spatial_integrals."""
    O, area, Lmax, x = block_geometry(mesh, j, l_in, l_out, d)
    a = np.where(area > 0.0, mu * Lmax, 0.0)
    L = np.where(area > 0.0, Lmax, 0.0)
    A_in, A_out = mesh.area[j, l_in], mesh.area[j, l_out]
    dI = lambda i, m, aa: -moment_I(i + 1, m, aa)          # noqa: E731
    if pos_order == 0:
        return (2.0 * area * dI(0, 1, a) * L / math.sqrt(A_in * A_out))[:, None, None]
    from .geometry import barycentric_3d
    Q = d.shape[0]
    V = mesh.verts[mesh.fverts[j, l_in]]
    y, z = (x + 1) % 3, (x + 2) % 3
    b_in = _inbound_corner_basis(mesh, j, l_in, x, O, 1)
    Fv = mesh.verts[mesh.fverts[j, l_out]]
    E = O @ V + L[:, None] * d
    imgs = np.stack([E, np.broadcast_to(V[y], E.shape), np.broadcast_to(V[z], E.shape)], axis=1)
    lam_out = barycentric_3d(imgs.reshape(-1, 3), Fv[0], Fv[1], Fv[2]).reshape(Q, 3, 3)
    b_out = basis.position_basis(lam_out, A_out, 1)
    G = _corner_moments(dI, area, a) * L[:, None, None]
    return np.einsum("qap,qab,qbr->qpr", b_out, G, b_in)


def dB_dmu_block(mesh, bs: Basis, mu_j, j, l_in, l_out):
    """d(block)/d mu_j, same layout and normalisation as assemble.block."""
    d, W = quadrature.block_nodes(mesh, j, l_in, l_out, bs.quad_n, bs.rule)
    dS = dS_dmu(mesh, j, l_in, l_out, d, mu_j, bs.pos_order)
    slot, transmitted, weight, dframe = destination(mesh, j, l_out)
    n = mesh.n_out[j, l_out]
    d_dest = d if transmitted else d - 2.0 * np.outer(d @ n, n)
    ci, pi_ = basis.direction_angles(d, mesh.frame[j, l_in])
    co, po = basis.direction_angles(d_dest, dframe)
    psi = basis.momentum(ci, pi_, bs.mom_degree, bs.mom_family)
    psi_o = basis.momentum(co, po, bs.mom_degree, bs.mom_family)
    T = np.einsum("q,qab,qk,ql->akbl", W, dS, psi_o, psi, optimize=True).reshape(bs.K, bs.K)
    G = basis.gram(bs.mom_degree, bs.mom_family)
    out = np.empty_like(T)
    M = bs.M
    for p in range(bs.P):
        out[p * M:(p + 1) * M] = np.linalg.solve(G, T[p * M:(p + 1) * M])
    return weight * out, slot


def gradient_mu(mesh, bs: Basis, mu, lam, rho, box):
    """dJ/dmu_e = lambda^T dB/dmu_e rho + dg/dmu_e . rho for every tet e."""
    K = bs.K
    lam = lam.reshape(4 * mesh.nt, K)
    rr = rho.reshape(4 * mesh.nt, K)
    out = np.zeros(mesh.nt)
    for j in range(mesh.nt):
        for l_out in range(4):
            for l_in in in_faces(l_out):
                dB, slot = dB_dmu_block(mesh, bs, mu[j], j, l_in, l_out)
                out[j] += lam[slot] @ dB @ rr[4 * j + l_in]
    dg = receiver_functional(mesh, bs, mu, box, derivative=True).reshape(mesh.nt, -1)
    out += np.einsum("jk,jk->j", dg, rho.reshape(mesh.nt, -1))
    return out
