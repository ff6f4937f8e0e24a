"""Seeded synthetic inputs for discrete flow mapping on tetrahedral meshes.

This module only *describes* problems: box meshes split into tetrahedra,
per-element damping fields, boundary reflection coefficients and source
descriptions.  It contains none of the method's arithmetic (no face matching,
no frames, no quadrature, no basis functions), so both the CPU oracle and the
GPU library can be driven from the same inputs without sharing code.

The paper's own meshes (a 972-tetrahedron cuboid, Sec. 4.1, and an industrial
1300-tetrahedron vehicle cavity, Sec. 4.2) are not available; structured,
jittered Kuhn/Freudenthal boxes stand in for them.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "kuhn_box",
    "Problem",
    "problem_c1",
    "problem_c2",
    "problem_c3",
    "problem_c5",
    "uniform_points_on_box_surface",
]

# The six tetrahedra of one cube cell: corner 0 -> e_a -> e_a + e_b -> (1,1,1)
# for every permutation (a, b, c) of the three axes.
_PERMS = list(itertools.permutations((0, 1, 2)))


def _vid(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def _signed_volumes(verts, tets):
    p = verts[tets]
    a = p[:, 1] - p[:, 0]
    b = p[:, 2] - p[:, 0]
    c = p[:, 3] - p[:, 0]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def kuhn_box(n=(1, 1, 1), size=(1.0, 1.0, 1.0), jitter=0.0, seed=None):
    """Structured box [0,Lx]x[0,Ly]x[0,Lz] with nx*ny*nz cells, 6 tets per cell.

    Vertex (i, j, k) has index i + (nx+1)*(j + (ny+1)*k).  Tetrahedra of cell
    (i, j, k) are listed in the order of ``itertools.permutations((0,1,2))``.

    ``jitter`` is a fraction of the cell size h (per axis): interior vertices
    move by U(-jitter*h, jitter*h) in all three coordinates, boundary vertices
    only in the coordinates that are not pinned to a box plane, so the box
    stays a box.  If a draw inverts or flattens a tetrahedron the whole field is
    redrawn from the same generator (deterministic for a given seed).
    """
    nx, ny, nz = (int(v) for v in n)
    lx, ly, lz = (float(v) for v in size)
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # flatten in vertex-index order (i fastest)
    ii = ii.transpose(2, 1, 0).ravel()
    jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    # i * L / n (not i * h) so that the last grid plane sits exactly on L
    grid = np.stack([ii * lx / nx, jj * ly / ny, kk * lz / nz], axis=1).astype(np.float64)

    tets = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for perm in _PERMS:
                    c = [i, j, k]
                    ids = [_vid(c[0], c[1], c[2], nx, ny)]
                    for ax in perm:
                        c[ax] += 1
                        ids.append(_vid(c[0], c[1], c[2], nx, ny))
                    tets.append(ids)
    tets = np.asarray(tets, dtype=np.int64)
    verts = grid.copy()
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        free = np.stack([(ii > 0) & (ii < nx), (jj > 0) & (jj < ny), (kk > 0) & (kk < nz)], axis=1)
        h = np.array([hx, hy, hz])
        vol0 = _signed_volumes(grid, tets)
        for _attempt in range(100):
            disp = rng.uniform(-jitter, jitter, size=grid.shape) * h
            verts = grid + np.where(free, disp, 0.0)
            vol = _signed_volumes(verts, tets)
            if np.all(vol * np.sign(vol0) > 1e-3 * np.abs(vol0)):
                break
        else:  # pragma: no cover - never reached for jitter <= 0.25
            raise RuntimeError("could not draw a valid jittered mesh")
    return verts, tets


def face_vertices(tets):
    """Global vertex ids of face l of every tet (face l is opposite local vertex l)."""
    out = np.empty((tets.shape[0], 4, 3), dtype=tets.dtype)
    for l in range(4):
        out[:, l, :] = tets[:, [m for m in range(4) if m != l]]
    return out


def uniform_points_on_box_surface(size, count, rng):
    """Points uniform by area on the surface of the box [0,Lx]x[0,Ly]x[0,Lz]."""
    lx, ly, lz = size
    areas = np.array([ly * lz, ly * lz, lx * lz, lx * lz, lx * ly, lx * ly])
    side = rng.choice(6, size=count, p=areas / areas.sum())
    u = rng.uniform(size=count)
    v = rng.uniform(size=count)
    pts = np.empty((count, 3))
    for s in range(6):
        m = side == s
        ax = s // 2
        other = [a for a in range(3) if a != ax]
        pts[m, ax] = 0.0 if s % 2 == 0 else size[ax]
        pts[m, other[0]] = u[m] * size[other[0]]
        pts[m, other[1]] = v[m] * size[other[1]]
    return pts


@dataclass
class Problem:
    """A complete synthetic DFM problem description (all host numpy arrays)."""

    name: str
    verts: np.ndarray            # [nv][3] f64
    tets: np.ndarray             # [nt][4] i64
    mu: np.ndarray               # [nt] damping per unit length
    refl: np.ndarray             # [nt][4] reflection coefficient of face l (used on boundary faces only)
    pos_order: int               # 0: piecewise constant, 1: piecewise linear per face
    mom_degree: int              # total degree D of the momentum basis
    quad_n: int                  # Gauss-Legendre points per dimension per cell
    source: dict = field(default_factory=dict)
    size: tuple = (1.0, 1.0, 1.0)

    @property
    def nt(self):
        return int(self.tets.shape[0])


def _refl_field(verts, tets, wall, absorbing_plane=None):
    """Reflection coefficient per (tet, face); faces lying in ``absorbing_plane``
    (axis, value) get 0.  Interior faces carry a value too but it is never used."""
    refl = np.full((tets.shape[0], 4), float(wall))
    if absorbing_plane is not None:
        ax, val = absorbing_plane
        fv = face_vertices(tets)
        on = np.all(verts[fv][..., ax] == val, axis=-1)
        refl[on] = 0.0
    return refl


def problem_c1():
    """Unit cube, 6 Kuhn tets, P0 x Legendre D=4, 8-point GL, mu=0.

    Walls reflect fully except the face x=1 (R=0); source: unit flux,
    cos(theta)-weighted, uniform over the face x=0."""
    verts, tets = kuhn_box((1, 1, 1), (1.0, 1.0, 1.0))
    return Problem(
        name="cube6_p0_d4_n8",
        verts=verts,
        tets=tets,
        mu=np.zeros(tets.shape[0]),
        refl=_refl_field(verts, tets, 1.0, absorbing_plane=(0, 1.0)),
        pos_order=0,
        mom_degree=4,
        quad_n=8,
        source={"kind": "face_flux", "axis": 0, "value": 0.0, "flux": 1.0},
    )


def problem_c2(n_cells=8, seed=0):
    """Box [0,1]^3 with 8^3 cells (3072 tets), jitter 0.15h, P1 x Legendre D=8,
    12-point GL, mu=0.05, walls R=0.9, Gaussian patch source on x=0."""
    verts, tets = kuhn_box((n_cells,) * 3, (1.0, 1.0, 1.0), jitter=0.15, seed=seed)
    return Problem(
        name=f"box{n_cells}_p1_d8_n12",
        verts=verts,
        tets=tets,
        mu=np.full(tets.shape[0], 0.05),
        refl=_refl_field(verts, tets, 0.9),
        pos_order=1,
        mom_degree=8,
        quad_n=12,
        source={"kind": "gauss_patch", "axis": 0, "value": 0.0, "center": (0.0, 0.5, 0.5),
                "sigma": 0.1, "flux": 1.0},
    )


def problem_c3(cells=(32, 16, 16), nsrc=128, seeds=(1, 2, 3)):
    """Box 2x1x1 with 32x16x16 cells (49152 tets), jitter 0.1h, P0 x Legendre
    D=12, mu lognormal(ln 0.02, 0.5) per element, walls R=0.9, ``nsrc`` isotropic
    point sources uniform by area on the boundary."""
    size = (2.0, 1.0, 1.0)
    verts, tets = kuhn_box(cells, size, jitter=0.1, seed=seeds[0])
    mu = np.random.default_rng(seeds[1]).lognormal(np.log(0.02), 0.5, size=tets.shape[0])
    pts = uniform_points_on_box_surface(size, nsrc, np.random.default_rng(seeds[2]))
    return Problem(
        name="box32x16x16_p0_d12_n16",
        verts=verts,
        tets=tets,
        mu=mu,
        refl=_refl_field(verts, tets, 0.9),
        pos_order=0,
        mom_degree=12,
        quad_n=16,
        source={"kind": "points", "xyz": pts, "flux": 1.0},
        size=size,
    )


def problem_c5(n_instances=256, seed=5, tets_range=(500, 20000)):
    """Uneven batch: ``n_instances`` independent boxes (1, U[1,4], U[1,4]) with a
    log-uniform target tet count T in ``tets_range``, cells n_i = max(1, round(L_i
    (T / (6 L_x L_y L_z))^(1/3))), jitter 0.2h; per box mu ~ U[0, 0.1] (uniform
    over the box), walls R = 0.9, P0 x Legendre of degree uniform in {4, 6, 8, 10}
    with n = D + 4 Gauss points, 4 isotropic point sources uniform by area on its
    boundary.  Each box is its own Problem; seeds derive from ``seed``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_instances):
        size = (1.0, float(rng.uniform(1.0, 4.0)), float(rng.uniform(1.0, 4.0)))
        T = float(np.exp(rng.uniform(np.log(tets_range[0]), np.log(tets_range[1]))))
        h = (T / (6.0 * size[0] * size[1] * size[2])) ** (1.0 / 3.0)
        cells = tuple(max(1, int(round(L * h))) for L in size)
        D = int(rng.choice([4, 6, 8, 10]))
        mu_i = float(rng.uniform(0.0, 0.1))
        verts, tets = kuhn_box(cells, size, jitter=0.2, seed=int(rng.integers(1 << 31)))
        pts = uniform_points_on_box_surface(size, 4, np.random.default_rng(int(rng.integers(1 << 31))))
        out.append(Problem(
            name=f"uneven{i}_{cells[0]}x{cells[1]}x{cells[2]}_p0_d{D}",
            verts=verts,
            tets=tets,
            mu=np.full(tets.shape[0], mu_i),
            refl=_refl_field(verts, tets, 0.9),
            pos_order=0,
            mom_degree=D,
            quad_n=D + 4,
            source={"kind": "points", "xyz": pts, "flux": 1.0},
            size=size,
        ))
    return out

