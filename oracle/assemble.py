"""Galerkin matrix B of the weighted boundary operator (paper Sec. 3.2, Eq. Bapprox / B4DInt).

One block maps the coefficients of the density entering tet j through face
l_in to the coefficients of the density that, after crossing tet j and leaving
through face l_out, enters the destination slot (the neighbour's copy of the
face, or tet j's own face after a wall reflection):

  T[(p',k'),(p,k)] = sum_q W_q S_q[p',p] psi'_k'(d'_q) psi_k(d_q)
  B_block = w * (I_P kron G^{-1}) T

with W_q the direction weight (flux measure), S the analytic spatial integral
(geometry.py), psi / psi' the momentum basis in the inbound / destination face
frame (step 4 of the five steps: d' = d on transmission, the specular image on
reflection), w the transmission (1) or reflection (R) weight, and G the Gram
matrix of the momentum family.  For the Zernike family G^{-1} is the factor
(2n'+2)/(eps_m' pi) of Eq. Bapprox.

Storage: B[j][l_out][s][K][K] where s runs over l_in in increasing order with
l_in != l_out, and dest[j][l_out] is the destination slot 4*i + l''.
The global unknown vector is indexed [slot][p][k], slot = 4*tet + face.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import basis, geometry, quadrature
from .mesh import destination


@dataclass
class Basis:
    pos_order: int = 0
    mom_family: int = basis.LEGENDRE
    mom_degree: int = 4
    quad_n: int = 8
    rule: int = quadrature.PAPER_RULE

    @property
    def P(self):
        return basis.position_count(self.pos_order)

    @property
    def M(self):
        return basis.momentum_count(self.mom_degree)

    @property
    def K(self):
        return self.P * self.M


def in_faces(l_out):
    return [l for l in range(4) if l != l_out]


def block_T(mesh, bs, mu_j, j, l_in, l_out):
    """Unnormalised block T, destination slot and weight."""
    d, W = quadrature.block_nodes(mesh, j, l_in, l_out, bs.quad_n, bs.rule)
    S = geometry.spatial_integrals(mesh, j, l_in, l_out, d, mu_j, bs.pos_order)
    slot, transmitted, weight, dframe = destination(mesh, j, l_out)
    if transmitted:
        d_dest = d
    else:
        n = mesh.n_out[j, l_out]
        d_dest = d - 2.0 * np.outer(d @ n, n)
    ci, pi_ = basis.direction_angles(d, mesh.frame[j, l_in])
    co, po = basis.direction_angles(d_dest, dframe)
    psi = basis.momentum(ci, pi_, bs.mom_degree, bs.mom_family)
    psi_o = basis.momentum(co, po, bs.mom_degree, bs.mom_family)
    T = np.einsum("q,qab,qk,ql->akbl", W, S, psi_o, psi, optimize=True)
    P, M = bs.P, bs.M
    return T.reshape(P * M, P * M), slot, weight


def block(mesh, bs, mu_j, j, l_in, l_out):
    T, slot, weight = block_T(mesh, bs, mu_j, j, l_in, l_out)
    G = basis.gram(bs.mom_degree, bs.mom_family)
    P, M = bs.P, bs.M
    B = np.empty_like(T)
    for p in range(P):
        B[p * M:(p + 1) * M] = np.linalg.solve(G, T[p * M:(p + 1) * M])
    return weight * B, slot


def assemble(mesh, bs, mu, tets=None):
    """Blocks of the listed tets (default all): B [len][4][3][K][K], dest [len][4]."""
    tets = range(mesh.nt) if tets is None else list(tets)
    K = bs.K
    out = np.zeros((len(tets), 4, 3, K, K))
    dest = np.zeros((len(tets), 4), dtype=np.int64)
    for t, j in enumerate(tets):
        for l_out in range(4):
            for s, l_in in enumerate(in_faces(l_out)):
                out[t, l_out, s], dest[t, l_out] = block(mesh, bs, mu[j], j, l_in, l_out)
    return out, dest
