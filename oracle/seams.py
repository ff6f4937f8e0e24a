"""Cells that keep the momentum-basis integrand smooth (a rule the paper does not need).

The paper's Zernike basis is smooth on the whole hemisphere (it vanishes at
theta = 0 for m != 0 and is periodic in phi, Sec. 3.4), so its integrand is
smooth inside each of the seven regions.  A tensor Legendre basis in
(cos theta, phi/pi) is not: it jumps across the half-plane phi = 0 of its
frame and depends on phi at theta = 0.  Both happen twice per block, for the
inbound frame (basis psi(d)) and for the destination frame (basis psi'(d')).

Rule (applied to every region that reaches the outbound face, in region order):
 1. cut by the planes through the inbound pole z_in normal to the inbound y
    axis (the seam phi = 0 lies in it) and normal to the inbound x axis;
 2. cut by the planes normal to the destination frame's y and x axes (they
    contain the direction n_F whose image d' is the destination pole: d' = d
    for transmission, and a reflection fixes the in-face axes, so the seams of
    both cases are the same great circle);
 3. cut by the bisector plane normal to z_in - n_F, which puts the two poles
    in different cells;
 every cut keeps the positive side first, then the negative side.  After
 steps 1-2 every cell that touches a pole lies in one quadrant around it, so
 phi of that frame varies by at most pi/2 over the cell;
 4. a cell with a pole on its boundary is fanned into triangles from the pole
    (the pole is the collapsed vertex v1 = v4 of the patch map, so phi of that
    frame depends on one patch coordinate only); a cell without a pole is used
    as a triangle or quadrilateral if it has 3 or 4 corners, else fanned from
    its first corner.
Every on-plane / on-edge / same-vertex decision uses the absolute tolerance
TOL on unit vectors.
"""
from __future__ import annotations

import numpy as np

TOL = 1e-12


def _unit(v):
    return v / np.linalg.norm(v)


def _polygon(patch):
    """Corner list of a patch (drops the repeated v4 = v1 of a triangle)."""
    pts = [np.asarray(p, dtype=np.float64) for p in patch]
    out = []
    for p in pts:
        if not out or np.linalg.norm(p - out[-1]) > TOL:
            out.append(p)
    if len(out) > 1 and np.linalg.norm(out[0] - out[-1]) <= TOL:
        out.pop()
    return out


def clip(poly, nrm):
    """Split a convex spherical polygon by the great circle normal to nrm.

    Returns (positive part, negative part); a part with no corner strictly on
    its side is None."""
    m = len(poly)
    s = [float(v @ nrm) for v in poly]
    pos, neg = [], []
    for k in range(m):
        a, b = poly[k], poly[(k + 1) % m]
        sa, sb = s[k], s[(k + 1) % m]
        if sa >= -TOL:
            pos.append(a)
        if sa <= TOL:
            neg.append(a)
        if (sa > TOL and sb < -TOL) or (sa < -TOL and sb > TOL):
            p = _unit((sa * b - sb * a) / (sa - sb))
            pos.append(p)
            neg.append(p)
    keep_pos = any(v > TOL for v in s) and len(pos) >= 3
    keep_neg = any(v < -TOL for v in s) and len(neg) >= 3
    return (pos if keep_pos else None), (neg if keep_neg else None)


def _locate(poly, p):
    """('vertex', k) | ('edge', k) | ('inside', -1) | None for a point p on the sphere."""
    m = len(poly)
    for k in range(m):
        if np.linalg.norm(poly[k] - p) <= TOL:
            return ("vertex", k)
    centre = np.sum(poly, axis=0)                 # inside a convex spherical polygon
    on_edge = -1
    for k in range(m):
        nrm = np.cross(poly[k], poly[(k + 1) % m])
        nrm = nrm / np.linalg.norm(nrm)
        if nrm @ centre < 0.0:
            nrm = -nrm
        e = nrm @ p
        if e < -TOL:
            return None
        if e <= TOL and on_edge < 0:
            on_edge = k
    if on_edge >= 0:
        return ("edge", on_edge)
    return ("inside", -1)


def _fan(poly, poles):
    m = len(poly)
    for p in poles:
        where = _locate(poly, p)
        if where is None:
            continue
        kind, k = where
        if kind == "vertex":
            ring = poly[k:] + poly[:k]
            return [np.array([ring[0], ring[i], ring[i + 1], ring[0]]) for i in range(1, m - 1)]
        if kind == "edge":
            ring = [p] + poly[k + 1:] + poly[:k + 1]
            return [np.array([p, ring[i], ring[i + 1], p]) for i in range(1, len(ring) - 1)]
        return [np.array([p, poly[i], poly[(i + 1) % m], p]) for i in range(m)]
    if m == 3:
        return [np.array([poly[0], poly[1], poly[2], poly[0]])]
    if m == 4:
        return [np.array(poly)]
    return [np.array([poly[0], poly[i], poly[i + 1], poly[0]]) for i in range(1, m - 1)]


def cut_cells(mesh, j, l_in, l_out, regions):
    x_in, y_in, z_in = mesh.frame[j, l_in]
    n_f = mesh.n_out[j, l_out]
    slot = mesh.nbr[j, l_out]
    dest_frame = mesh.frame[slot // 4, slot % 4] if slot >= 0 else mesh.frame[j, l_out]
    planes = [y_in, x_in, dest_frame[1], dest_frame[0], z_in - n_f]
    polys = [_polygon(r) for r in regions]
    for nrm in planes:
        nxt = []
        for poly in polys:
            pos, neg = clip(poly, nrm)
            if pos is not None:
                nxt.append(pos)
            if neg is not None:
                nxt.append(neg)
        polys = nxt
    cells = []
    for poly in polys:
        cells.extend(_fan(poly, [z_in, n_f]))
    return cells
