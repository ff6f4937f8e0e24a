"""Direction-space quadrature (paper Sec. 3.4).

The inward hemisphere of an inbound face ABC (apex D) is split into the seven
sub-regions of Sec. 3.3/3.4, one for each possible location of the point O.
Each sub-region is a spherical triangle or quadrilateral whose sides are the
great circles that separate the regions plus the equator; it is mapped from
[-1,1]^2 by the bilinear patch of Eq. Parametr followed by the radial
projection g = f/|f|, with the Jacobian of Sec. 3.4 (which already contains the
sin(2 theta)/2 = cos(theta) sin(theta) factor of Eq. B4DInt).  A tensor
Gauss-Legendre rule with n points per dimension is used on every patch; the
paper uses adaptive Clenshaw-Curtis instead (Sec. 3.4), a fixed Gauss rule is
the configuration this implementation is measured on.

The seven regions, for base vertices A, B, C in increasing global id and with
d_XD = unit(D - X), u(V) = unit(V):
  0      central triangle (d_AD, d_BD, d_CD)           -> all three outbound faces
  1+x    quadrilateral beyond edge X-Y (Y = x+1, Z = x+2 mod 3):
         (d_XD, d_YD, u(Z-Y), u(Z-X))                   -> faces F_X and F_Y
  4+x    triangle at vertex X: (d_XD, u(Y-X), u(Z-X))   -> face F_X only
where F_X is the outbound face opposite base vertex X.  These are the regions
of Fig. xyCircles: P inside ABC, P beyond one edge, P in a vertex wedge.
Triangles are patches with v4 = v1.
"""
from __future__ import annotations

import numpy as np

from . import seams

PAPER_RULE = 0
SEAM_RULE = 1


def gauss_legendre(n):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _unit(v):
    return v / np.linalg.norm(v)


def base_and_apex(mesh, j, l_in):
    """Base vertices (A, B, C) of inbound face l_in in increasing global id, the
    apex D, and for each base vertex X the local index of the outbound face F_X."""
    ids = mesh.fverts[j, l_in]
    A, B, C = (mesh.verts[g] for g in ids)
    D = mesh.verts[mesh.tets[j, l_in]]
    out_face = [int(np.nonzero(mesh.tets[j] == g)[0][0]) for g in ids]
    return (A, B, C), D, out_face


def seven_pieces(mesh, j, l_in):
    """The seven direction sub-regions of inbound face l_in of tet j.

    Returns a list of (patch [4][3], reachable outbound local faces)."""
    V, D, out_face = base_and_apex(mesh, j, l_in)
    dD = [_unit(D - X) for X in V]
    pieces = [(np.array([dD[0], dD[1], dD[2], dD[0]]), set(out_face))]
    for x in range(3):
        y, z = (x + 1) % 3, (x + 2) % 3
        quad = np.array([dD[x], dD[y], _unit(V[z] - V[y]), _unit(V[z] - V[x])])
        pieces.append((quad, {out_face[x], out_face[y]}))
    for x in range(3):
        y, z = (x + 1) % 3, (x + 2) % 3
        tri = np.array([dD[x], _unit(V[y] - V[x]), _unit(V[z] - V[x]), dD[x]])
        pieces.append((tri, {out_face[x]}))
    return pieces


def block_cells(mesh, j, l_in, l_out, rule=PAPER_RULE):
    """Quadrature cells (patches [4][3]) for the block (inbound l_in -> outbound l_out).

    PAPER_RULE: the four of the seven regions from which face l_out is reachable,
    in region order.  SEAM_RULE: those regions further cut where the momentum
    basis is not smooth (see ``seams``)."""
    cells = [p for (p, reach) in seven_pieces(mesh, j, l_in) if l_out in reach]
    if rule == PAPER_RULE:
        return cells
    return seams.cut_cells(mesh, j, l_in, l_out, cells)


def patch_nodes(patch, xg, wg, z_in):
    """Directions and weights of the n x n Gauss rule on one patch.

    f = a + b xi + c eta + d xi eta (Eq. Parametr), g = f/|f|,
    weight = w_xi w_eta * (f . z_in) |det[f, f_xi, f_eta]| / |f|^4 (Sec. 3.4;
    the absolute value of the determinant is taken, the paper prints none)."""
    v1, v2, v3, v4 = patch
    a = 0.25 * (v1 + v2 + v3 + v4)
    b = 0.25 * (v2 - v1 + v3 - v4)
    c = 0.25 * (v3 + v4 - v1 - v2)
    d = 0.25 * (v3 - v4 + v1 - v2)
    xi = np.repeat(xg, len(xg))
    eta = np.tile(xg, len(xg))
    w = np.repeat(wg, len(wg)) * np.tile(wg, len(wg))
    f = a + np.outer(xi, b) + np.outer(eta, c) + np.outer(xi * eta, d)
    f_xi = b + np.outer(eta, d)
    f_eta = c + np.outer(xi, d)
    det = np.einsum("qi,qi->q", f, np.cross(f_xi, f_eta))
    nf = np.linalg.norm(f, axis=1)
    jac = (f @ z_in) * np.abs(det) / nf ** 4
    return f / nf[:, None], w * jac


def block_nodes(mesh, j, l_in, l_out, n, rule=PAPER_RULE):
    """All quadrature directions [Q,3] and weights [Q] of one block."""
    xg, wg = gauss_legendre(n)
    z_in = mesh.frame[j, l_in, 2]
    ds, ws = [], []
    for patch in block_cells(mesh, j, l_in, l_out, rule):
        d, w = patch_nodes(patch, xg, wg, z_in)
        ds.append(d)
        ws.append(w)
    return np.concatenate(ds), np.concatenate(ws)
