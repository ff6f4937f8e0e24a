"""Steps 1-3 of the five steps of Sec. 3.3 for one (inbound face, outbound face) pair.

For a direction d entering tet ABCD through its face ABC (local frame of that
face: origin A, x along AB, z the inward normal, so D = (D1, D2, D3), D3 > 0):

 1. the point P of the xy-plane with P -> D parallel to d is
    P = (D1, D2) - D3 tan(theta) (cos phi, sin phi); the three extended edges
    of ABC split the plane into seven regions, told apart here by the signs of
    P's barycentric coordinates.  O = P inside ABC; beyond one edge, O is the
    point where the line from the opposite vertex through P meets that edge;
    in a vertex wedge, O is that vertex (Fig. xyCircles).  The set of start
    points whose rays reach the outbound face F_X (opposite base vertex X) is
    the triangle O Y Z spanned by O and F_X's edge Y Z on ABC; it is empty
    when O lies on that edge.
 2. L_max is the length of the ray from O along d until it leaves the tet.
 3. the chord length is linear on O Y Z, L_max at O and 0 on Y Z, so
    int_{OYZ} exp(-mu L) ds = h |YZ| (mu L_max - 1 + exp(-mu L_max)) / (mu L_max)^2
    with h|YZ|/2 the area of OYZ (the formula of Sec. 3.3); it is that area for
    mu = 0.

For the piecewise-linear position basis the same linearity gives the integral
of b'(exit point) b(start point) exp(-mu L) over OYZ from the moments
int_T l_O^i l_Y^j l_Z^k exp(-a l_O) dA = 2|T| j! k!/(j+k+1)! I_{i,j+k+1}(a),
I_{i,m}(a) = int_0^1 u^i (1-u)^m exp(-a u) du = B(i+1, m+1) 1F1(i+1; i+m+2; -a),
because the exit map s -> s + L(s) d is affine on OYZ (it fixes Y and Z and
sends O to O + L_max d) and both position bases are affine on their faces.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import hyp1f1

from . import basis
from .quadrature import base_and_apex


def g_exp(a):
    """(a - 1 + exp(-a)) / a^2, the paper's closed form divided by h|BC|.

    Evaluated as (a + expm1(-a))/a^2 for a >= 0.1 and by its Taylor series
    sum_r (-a)^r / (r+2)! below, where the closed form cancels."""
    a = np.asarray(a, dtype=np.float64)
    big = a >= 0.1
    ab = np.where(big, a, 1.0)
    closed = (ab + np.expm1(-ab)) / (ab * ab)
    series = np.zeros_like(a)
    term = np.full_like(a, 0.5)              # (-a)^0 / 2!
    for r in range(20):
        series = series + term
        term = term * (-a) / (r + 3)
    return np.where(big, closed, series)


def moment_I(i, m, a):
    """I_{i,m}(a) = int_0^1 u^i (1-u)^m exp(-a u) du."""
    beta = math.factorial(i) * math.factorial(m) / math.factorial(i + m + 1)
    return beta * hyp1f1(i + 1, i + m + 2, -np.asarray(a, dtype=np.float64))


def barycentric_2d(P, A, B, C):
    """Barycentric coordinates [Q,3] of 2-D points P [Q,2] in triangle ABC."""
    T = np.array([[B[0] - A[0], C[0] - A[0]], [B[1] - A[1], C[1] - A[1]]])
    lb, lc = np.linalg.solve(T, (P - A).T)
    return np.stack([1.0 - lb - lc, lb, lc], axis=1)


def barycentric_3d(q, v0, v1, v2):
    """Barycentric coordinates of points q [Q,3] lying in the plane of v0 v1 v2."""
    n = np.cross(v1 - v0, v2 - v0)
    nn = n @ n
    l1 = np.einsum("qi,i->q", np.cross(q - v0, v2 - v0), n) / nn
    l2 = np.einsum("qi,i->q", np.cross(v1 - v0, q - v0), n) / nn
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1)


def point_O(lam):
    """Barycentric coordinates of O from those of P (rule of Sec. 3.3)."""
    O = np.array(lam, copy=True)
    neg = lam < 0.0
    cnt = neg.sum(axis=1)
    # beyond one edge: project along the line from the opposite vertex
    one = cnt == 1
    if np.any(one):
        l1 = np.where(neg[one], 0.0, lam[one])
        O[one] = l1 / l1.sum(axis=1, keepdims=True)
    # in a vertex wedge: the vertex itself
    two = cnt == 2
    if np.any(two):
        O[two] = np.where(neg[two], 0.0, 1.0)
    return O


def block_geometry(mesh, j, l_in, l_out, d):
    """Per-direction region data for block (l_in -> l_out): barycentric O [Q,3],
    the area of the start set OYZ [Q], L_max [Q], and the index x of the base
    vertex opposite the outbound face."""
    (A, B, C), D, out_face = base_and_apex(mesh, j, l_in)
    x = out_face.index(l_out)
    V = np.stack([A, B, C])
    fr = mesh.frame[j, l_in]
    loc = lambda v: fr @ (v - A)                       # noqa: E731
    A2, B2, C2, Dl = np.zeros(2), loc(B)[:2], loc(C)[:2], loc(D)
    dl = d @ fr.T
    P = Dl[:2][None, :] - (Dl[2] / dl[:, 2])[:, None] * dl[:, :2]
    O = point_O(barycentric_2d(P, A2, B2, C2))
    Opos = O @ V
    Y, Z = V[(x + 1) % 3], V[(x + 2) % 3]
    area = 0.5 * np.linalg.norm(np.cross(Y - Opos, Z - Opos), axis=1)
    area = np.where(O[:, x] > 0.0, area, 0.0)
    # L_max: exit distance of the ray from O (nearest face plane it moves towards)
    Lmax = np.full(d.shape[0], np.inf)
    for g in range(4):
        ng = mesh.n_out[j, g]
        pg = mesh.verts[mesh.fverts[j, g, 0]]
        dn = d @ ng
        with np.errstate(divide="ignore", invalid="ignore"):
            dist = np.where(dn > 0.0, ((pg - Opos) @ ng) / dn, np.inf)
        Lmax = np.minimum(Lmax, dist)
    return O, area, Lmax, x


def spatial_integrals(mesh, j, l_in, l_out, d, mu, pos_order):
    """S[q, p', p] = int over the start set of b'_p'(exit) b_p(start) exp(-mu L) ds."""
    O, area, Lmax, x = block_geometry(mesh, j, l_in, l_out, d)
    a = mu * Lmax
    a = np.where(area > 0.0, a, 0.0)
    A_in = mesh.area[j, l_in]
    A_out = mesh.area[j, l_out]
    if pos_order == 0:
        S = 2.0 * area * g_exp(a) / math.sqrt(A_in * A_out)
        return S[:, None, None]
    Q = d.shape[0]
    ids_in = mesh.fverts[j, l_in]
    V = mesh.verts[ids_in]
    y, z = (x + 1) % 3, (x + 2) % 3
    # start-set corners (O, Y, Z): barycentric in the inbound face
    lam_in = np.zeros((Q, 3, 3))
    lam_in[:, 0, :] = O
    lam_in[:, 1, y] = 1.0
    lam_in[:, 2, z] = 1.0
    b_in = basis.position_basis(lam_in, A_in, 1)                     # [Q, corner, p]
    # their images on the outbound face: (O + L_max d, Y, Z)
    Fv = mesh.verts[mesh.fverts[j, l_out]]
    E = O @ V + np.where(area > 0.0, Lmax, 0.0)[:, None] * d
    imgs = np.stack([E, np.broadcast_to(V[y], E.shape), np.broadcast_to(V[z], E.shape)], axis=1)
    lam_out = barycentric_3d(imgs.reshape(-1, 3), Fv[0], Fv[1], Fv[2]).reshape(Q, 3, 3)
    b_out = basis.position_basis(lam_out, A_out, 1)                  # [Q, corner, p']
    # Gram of the corner barycentrics with the exponential weight (corner 0 = O)
    G = np.zeros((Q, 3, 3))
    for al in range(3):
        for be in range(3):
            e = [0, 0, 0]
            e[al] += 1
            e[be] += 1
            i, jj, kk = e
            G[:, al, be] = 2.0 * area * math.factorial(jj) * math.factorial(kk) \
                / math.factorial(jj + kk + 1) * moment_I(i, jj + kk + 1, a)
    return np.einsum("qap,qab,qbr->qpr", b_out, G, b_in)
