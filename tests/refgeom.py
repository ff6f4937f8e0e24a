"""Independent reference computations used to pin the oracle (no oracle code inside).

* ``face_frame``: the face-frame convention restated from vertex positions.
* ``trace``: straight-ray exit of a point/direction from a tetrahedron.
* ``mc_block``: Monte Carlo estimate of an unnormalised block
      T[(p',k'),(p,k)] = int_{F_in} int_{hemisphere} [exit via F] exp(-mu L)
                         b'_p'(s') psi'_k'(d') b_p(s) psi_k(d) cos(theta) dOmega ds
  with s uniform on the inbound face and d cosine-distributed.
* ``clip_integral``: the same spatial integral for one fixed direction by exact
  polygon clipping of the inbound face against the oblique projection of the
  outbound face, then a high-order triangle rule.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre


def unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def face_ids(tet, l):
    return sorted(int(tet[m]) for m in range(4) if m != l)


def face_frame(verts, tet, l):
    """(x, y, z) rows: origin at the lowest-id vertex, x to the next, z into the tet."""
    ids = face_ids(tet, l)
    v0, v1, v2 = verts[ids]
    apex = verts[tet[l]]
    n = unit(np.cross(v1 - v0, v2 - v0))
    if (apex - v0) @ n < 0:
        n = -n                                  # make it point to the apex (inward)
    x = unit(v1 - v0)
    return np.stack([x, np.cross(n, x), n])


def outward_normal(verts, tet, l):
    return -face_frame(verts, tet, l)[2]


def face_area(verts, tet, l):
    v0, v1, v2 = verts[face_ids(tet, l)]
    return 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))


def bary(verts, ids, q):
    v0, v1, v2 = verts[ids]
    n = np.cross(v1 - v0, v2 - v0)
    nn = n @ n
    l1 = (np.cross(q - v0, v2 - v0) @ n) / nn
    l2 = (np.cross(v1 - v0, q - v0) @ n) / nn
    return np.stack([1 - l1 - l2, l1, l2], axis=-1)


def pos_basis(lam, area, order):
    e0 = np.full(lam.shape[:-1], 1.0 / math.sqrt(area))
    if order == 0:
        return e0[..., None]
    return np.stack([e0, math.sqrt(6 / area) * (lam[..., 1] - lam[..., 0]),
                     math.sqrt(2 / area) * (3 * lam[..., 2] - 1)], axis=-1)


def legendre_basis(cos_t, phi, D):
    x = 2 * cos_t - 1
    y = phi / np.pi - 1
    cols = []
    for t in range(D + 1):
        for b in range(t + 1):
            a = t - b
            cols.append(math.sqrt(2 * a + 1) * eval_legendre(a, x) * math.sqrt(2 * b + 1) * eval_legendre(b, y))
    return np.stack(cols, axis=-1)


def angles(d, fr):
    c = d @ fr[2]
    phi = np.mod(np.arctan2(d @ fr[1], d @ fr[0]), 2 * np.pi)
    return c, phi


def trace(verts, tet, s, d):
    """Exit distance and exit face (local index) of rays s + t d, t > 0."""
    best = np.full(s.shape[0], np.inf)
    face = np.full(s.shape[0], -1)
    for g in range(4):
        n = outward_normal(verts, tet, g)
        p = verts[face_ids(tet, g)[0]]
        dn = d @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(dn > 1e-300, ((p - s) @ n) / dn, np.inf)
        t = np.where(t < -1e-12, np.inf, t)
        upd = t < best
        best = np.where(upd, t, best)
        face = np.where(upd, g, face)
    return best, face


def mc_block(verts, tet, l_in, l_out, mu, D, pos_order, nsamp, rng, dest_frame=None, reflect=False):
    """Monte Carlo mean and standard error of the block T (see module doc)."""
    fr_in = face_frame(verts, tet, l_in)
    ids_in = face_ids(tet, l_in)
    ids_out = face_ids(tet, l_out)
    A_in = face_area(verts, tet, l_in)
    A_out = face_area(verts, tet, l_out)
    V = verts[ids_in]
    r1, r2 = rng.uniform(size=nsamp), rng.uniform(size=nsamp)
    sq = np.sqrt(r1)
    lam = np.stack([1 - sq, sq * (1 - r2), sq * r2], axis=1)
    s = lam @ V
    # cosine-weighted directions (Malley): uniform disk lifted to the hemisphere
    u1, u2 = rng.uniform(size=nsamp), rng.uniform(size=nsamp)
    rad, ang = np.sqrt(u1), 2 * np.pi * u2
    loc = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.sqrt(1 - u1)], axis=1)
    d = loc @ fr_in
    L, face = trace(verts, tet, s, d)
    hit = face == l_out
    ex = s + L[:, None] * d
    n_out = outward_normal(verts, tet, l_out)
    if dest_frame is None:
        dest_frame = face_frame(verts, tet, l_out)
        reflect = True
    dd = d - 2 * (d @ n_out)[:, None] * n_out if reflect else d
    ci, pi_ = angles(d, fr_in)
    co, po = angles(dd, dest_frame)
    psi = legendre_basis(ci, pi_, D)
    psio = legendre_basis(co, po, D)
    bi = pos_basis(lam, A_in, pos_order)
    bo = pos_basis(bary(verts, ids_out, ex), A_out, pos_order)
    w = np.where(hit, np.exp(-mu * np.where(hit, L, 0.0)), 0.0) * A_in * np.pi
    P = bi.shape[1]
    M = psi.shape[1]
    U = (bo[:, :, None] * psio[:, None, :]).reshape(nsamp, P * M)
    Wv = (bi[:, :, None] * psi[:, None, :]).reshape(nsamp, P * M)
    X = np.einsum("q,qa,qb->ab", w, U, Wv) / nsamp
    X2 = np.einsum("q,qa,qb->ab", w * w, U * U, Wv * Wv) / nsamp
    se = np.sqrt(np.maximum(X2 - X * X, 0.0) / nsamp)
    return X, se


def _clip_poly(poly, a, b):
    """Keep the part of 2-D polygon poly on the left of the directed line a -> b."""
    out = []
    m = len(poly)
    side = lambda p: (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])  # noqa: E731
    for k in range(m):
        P, Q = poly[k], poly[(k + 1) % m]
        sp, sq = side(P), side(Q)
        if sp >= 0:
            out.append(P)
        if (sp >= 0) != (sq >= 0):
            t = sp / (sp - sq)
            out.append(P + t * (Q - P))
    return out


def _tri_rule(n=20):
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (x + 1), 0.5 * w
    U, Vv = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * (1 - U)
    l1 = U.ravel()
    l2 = (Vv * (1 - U)).ravel()
    return np.stack([1 - l1 - l2, l1, l2], axis=1), 2 * W.ravel()     # weights sum to 1 (x area)


def clip_integral(verts, tet, l_in, l_out, d, mu, pos_order):
    """S[p', p] for one direction d by exact clipping (module doc)."""
    fr = face_frame(verts, tet, l_in)
    ids_in = face_ids(tet, l_in)
    ids_out = face_ids(tet, l_out)
    o = verts[ids_in[0]]
    to2 = lambda p: np.array([(p - o) @ fr[0], (p - o) @ fr[1]])      # noqa: E731
    tri_in = [to2(verts[i]) for i in ids_in]
    # project the outbound face along -d onto the inbound plane
    dz = d @ fr[2]
    proj = []
    for i in ids_out:
        p = verts[i]
        h = (p - o) @ fr[2]
        proj.append(to2(p - (h / dz) * d))
    # orient both counter-clockwise
    def ccw(t):
        a = (t[1][0] - t[0][0]) * (t[2][1] - t[0][1]) - (t[1][1] - t[0][1]) * (t[2][0] - t[0][0])
        return t if a > 0 else [t[0], t[2], t[1]]
    tri_in, proj = ccw(tri_in), ccw(proj)
    poly = tri_in
    for k in range(3):
        if len(poly) < 3:
            break
        poly = _clip_poly(poly, proj[k], proj[(k + 1) % 3])
    P = 1 if pos_order == 0 else 3
    S = np.zeros((P, P))
    if len(poly) < 3:
        return S
    lam_ref, w_ref = _tri_rule()
    n_out = outward_normal(verts, tet, l_out)
    p_out = verts[ids_out[0]]
    A_in = face_area(verts, tet, l_in)
    A_out = face_area(verts, tet, l_out)
    for k in range(1, len(poly) - 1):
        t = np.array([poly[0], poly[k], poly[k + 1]])
        area = 0.5 * abs((t[1, 0] - t[0, 0]) * (t[2, 1] - t[0, 1]) - (t[1, 1] - t[0, 1]) * (t[2, 0] - t[0, 0]))
        pts2 = lam_ref @ t
        pts = o + pts2[:, :1] * fr[0] + pts2[:, 1:2] * fr[1]
        L = ((p_out - pts) @ n_out) / (d @ n_out)
        ex = pts + L[:, None] * d
        bi = pos_basis(bary(verts, ids_in, pts), A_in, pos_order)
        bo = pos_basis(bary(verts, ids_out, ex), A_out, pos_order)
        S += area * np.einsum("q,qa,qb->ab", w_ref * np.exp(-mu * L), bo, bi)
    return S
