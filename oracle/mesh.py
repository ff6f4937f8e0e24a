"""Mesh topology and per-face geometry (paper Sec. 2 and the local face frames of Sec. 3.3).

Conventions (the paper leaves them open, Sec. 3.3 only says the origin is "one
of the vertices" and the x-axis "one of the edges"):

* Face l of tetrahedron j is the face opposite its local vertex l.
* A face's vertices are taken in increasing global vertex id: v0 < v1 < v2.
  Its frame has origin v0, x = unit(v1 - v0), z = the unit normal pointing
  INTO the tetrahedron that owns this copy of the face, y = z cross x.
  Both tetrahedra sharing a face therefore agree on x; y and z flip.
* Two faces are the same face when their sorted vertex-id triples agree.
  A triple seen once is a boundary face, twice an interior face; three or more
  times is a non-manifold mesh and an error.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


class MeshError(ValueError):
    pass


@dataclass
class Mesh:
    verts: np.ndarray      # [nv][3]
    tets: np.ndarray       # [nt][4] global vertex ids
    nbr: np.ndarray        # [nt][4] slot 4*i+l'' of the other copy of the face, -1 on the boundary
    fverts: np.ndarray     # [nt][4][3] sorted global vertex ids of each face
    area: np.ndarray       # [nt][4]
    n_out: np.ndarray      # [nt][4][3] outward unit normal
    frame: np.ndarray      # [nt][4][3][3] rows x, y, z of the face frame (z inward)
    volume: np.ndarray     # [nt]
    refl: np.ndarray       # [nt][4] reflection coefficient (boundary faces)

    @property
    def nt(self):
        return self.tets.shape[0]


def build_mesh(verts, tets, refl=None):
    """Face adjacency, areas, normals, frames and volumes of a tetrahedral mesh."""
    verts = np.asarray(verts, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    nt = tets.shape[0]
    if not np.all(np.isfinite(verts)):
        raise MeshError("non-finite vertex coordinate")

    # --- adjacency: a face is identified by its sorted vertex triple -------------
    fverts = np.empty((nt, 4, 3), dtype=np.int64)
    for l in range(4):
        fverts[:, l, :] = np.sort(tets[:, [m for m in range(4) if m != l]], axis=1)
    owners = {}
    for j in range(nt):
        for l in range(4):
            owners.setdefault(tuple(fverts[j, l]), []).append((j, l))
    nbr = -np.ones((nt, 4), dtype=np.int64)
    for key, occ in owners.items():
        if len(occ) > 2:
            raise MeshError(f"face {key} is shared by {len(occ)} tetrahedra")
        if len(occ) == 2:
            (j, l), (i, m) = occ
            nbr[j, l] = 4 * i + m
            nbr[i, m] = 4 * j + l

    # --- volumes -----------------------------------------------------------------
    p = verts[tets]
    det = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    volume = np.abs(det) / 6.0
    if not np.all(volume > 0.0):
        raise MeshError("degenerate tetrahedron (zero volume)")

    # --- per-face geometry -----------------------------------------------------
    v0 = verts[fverts[..., 0]]
    v1 = verts[fverts[..., 1]]
    v2 = verts[fverts[..., 2]]
    apex = verts[tets]                      # local vertex l is the apex of face l
    cr = np.cross(v1 - v0, v2 - v0)
    twice_area = np.linalg.norm(cr, axis=-1)
    area = 0.5 * twice_area
    n = cr / twice_area[..., None]
    # orient outward: the apex must lie on the negative side
    inward = np.einsum("...i,...i->...", apex - v0, n) > 0.0
    n_out = np.where(inward[..., None], -n, n)
    ex = (v1 - v0) / np.linalg.norm(v1 - v0, axis=-1)[..., None]
    ez = -n_out
    ey = np.cross(ez, ex)
    frame = np.stack([ex, ey, ez], axis=-2)

    if refl is None:
        refl = np.ones((nt, 4))
    refl = np.asarray(refl, dtype=np.float64).reshape(nt, 4)
    return Mesh(verts=verts, tets=tets, nbr=nbr, fverts=fverts, area=area, n_out=n_out,
                frame=frame, volume=volume, refl=refl)


def destination(mesh, j, l_out):
    """Where a ray leaving tet j through face l_out enters next (Sec. 2, Sec. 3.3).

    With a uniform phase velocity and fluid density the acoustic transmission
    probability of Sec. 3.3 is 1 at every interior face (equal impedances, no
    refraction), so the ray crosses into the neighbour.  On the boundary it is
    reflected specularly back into tet j with the face's coefficient R.

    Returns (slot, transmitted, weight, frame) where frame (3x3 rows x,y,z) is
    the destination slot's face frame.
    """
    k = int(mesh.nbr[j, l_out])
    if k >= 0:
        return k, True, 1.0, mesh.frame[k // 4, k % 4]
    return 4 * j + l_out, False, float(mesh.refl[j, l_out]), mesh.frame[j, l_out]
