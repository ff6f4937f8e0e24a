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


def mc_energy(verts, tet, l, mu, D, pos_order, nsamp, rng):
    """Monte Carlo mean and standard error of
        E[p, k] = int_{face l} int_{hemisphere} b_p(s) psi_k(d) ell(s, d) cos(theta) dOmega ds,
        ell = (1 - exp(-mu L)) / mu  (L itself when mu = 0),
    L the chord from s along d to the exit.  This is the energy inside the tet
    carried by the density b_p psi_k entering through face l: along a ray the
    interior density integrated over the tet leaves int_0^L exp(-mu t) dt
    (Sec. 4.1, Eq. IntDens, integrated over the element).  Samples: s uniform
    on the face, d cosine-distributed, so the measure integrates to A pi."""
    fr = face_frame(verts, tet, l)
    ids = face_ids(tet, l)
    A = face_area(verts, tet, l)
    V = verts[ids]
    r1, r2 = rng.uniform(size=nsamp), rng.uniform(size=nsamp)
    sq = np.sqrt(r1)
    lam = np.stack([1 - sq, sq * (1 - r2), sq * r2], axis=1)
    s = lam @ V
    u1, u2 = rng.uniform(size=nsamp), rng.uniform(size=nsamp)
    rad, ang = np.sqrt(u1), 2 * np.pi * u2
    d = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.sqrt(1 - u1)], axis=1) @ fr
    L, _ = trace(verts, tet, s, d)
    ell = L if mu == 0.0 else -np.expm1(-mu * L) / mu
    c, phi = angles(d, fr)
    psi = legendre_basis(c, phi, D)
    b = pos_basis(lam, A, pos_order)
    F = (A * np.pi) * ell[:, None, None] * b[:, :, None] * psi[:, None, :]     # [n, P, M]
    mean = F.mean(axis=0)
    se = F.std(axis=0) / math.sqrt(nsamp)
    return mean, se


def _quad_rule_on_triangle(n=12):
    """Barycentrics [Q][3] and weights (summing to 1) of a rule on the reference
    triangle built by splitting it at the centroid into three quadrilaterals,
    each mapped bilinearly from [0,1]^2 with an n x n Gauss-Legendre product rule."""
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (x + 1), 0.5 * w
    U, Vv = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu).ravel()
    U, Vv = U.ravel(), Vv.ravel()
    E = np.eye(3)
    cen = np.full(3, 1.0 / 3.0)
    lam_all, w_all = [], []
    for k in range(3):
        a, b_, c = E[k], E[(k + 1) % 3], E[(k + 2) % 3]
        q = [a, 0.5 * (a + b_), cen, 0.5 * (a + c)]           # a quadrilateral of area 1/3 (x area)
        pts = (np.outer((1 - U) * (1 - Vv), q[0]) + np.outer(U * (1 - Vv), q[1])
               + np.outer(U * Vv, q[2]) + np.outer((1 - U) * Vv, q[3]))
        # Jacobian of the bilinear map in barycentric (area-fraction) units
        dU = np.outer(1 - Vv, q[1] - q[0]) + np.outer(Vv, q[2] - q[3])
        dV = np.outer(1 - U, q[3] - q[0]) + np.outer(U, q[2] - q[1])
        jac = np.abs(dU[:, 1] * dV[:, 2] - dU[:, 2] * dV[:, 1])   # 2-D area in the (l1, l2) chart
        lam_all.append(pts)
        w_all.append(W * jac * 2.0)                                # the reference triangle has area 1/2
    return np.concatenate(lam_all), np.concatenate(w_all)


def gauss_patch_moments(verts, ids, center, sigma, pos_order, levels=2, n=12):
    """int_face b_p(s) exp(-|s-c|^2/(2 sigma^2))/(2 pi sigma^2) ds for the position
    basis of the face with vertices ids (increasing global id), by recursive
    midpoint subdivision of the face into 4**levels triangles with the
    centroid-split Gauss rule on each."""
    V = verts[ids]
    A = 0.5 * np.linalg.norm(np.cross(V[1] - V[0], V[2] - V[0]))
    tris = [V]
    for _ in range(levels):
        nxt = []
        for T in tris:
            m01, m12, m20 = 0.5 * (T[0] + T[1]), 0.5 * (T[1] + T[2]), 0.5 * (T[2] + T[0])
            nxt += [np.array([T[0], m01, m20]), np.array([m01, T[1], m12]),
                    np.array([m20, m12, T[2]]), np.array([m01, m12, m20])]
        tris = nxt
    lam_ref, w_ref = _quad_rule_on_triangle(n)
    c = np.asarray(center, dtype=np.float64)
    out = 0.0
    for T in tris:
        pts = lam_ref @ T
        At = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
        dens = np.exp(-np.sum((pts - c) ** 2, axis=1) / (2 * sigma ** 2)) / (2 * np.pi * sigma ** 2)
        b = pos_basis(bary(verts, ids, pts), A, pos_order)
        out = out + (w_ref * At * dens) @ b
    return out
