"""Host logic of uneven batches (no GPU): grouping by discretisation, tet offsets,
and the placement of the instances of a group in one mesh.  The transport is
translation invariant, so every instance is moved by a constant vector; the
instances must not overlap, and every source point must stay on the boundary of
its own instance, or the point location of the library would find it on another
instance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from paper_1608_04607_amd.batch import UnevenBatch  # noqa: E402


def _on_box_surface(p, lo, hi, tol=1e-9):
    inside = np.all(p >= lo - tol, axis=1) & np.all(p <= hi + tol, axis=1)
    on_face = np.any(np.isclose(p, lo, atol=tol) | np.isclose(p, hi, atol=tol), axis=1)
    return inside & on_face


def test_grouping_offsets_and_placement():
    probs = synth.problem_c5(n_instances=40, seed=5, tets_range=(200, 1500))
    ub = UnevenBatch(probs, device="cpu")
    # every instance in exactly one group, groups keyed by their discretisation
    members = sorted(i for g in ub.groups for i in g.members)
    assert members == list(range(len(probs)))
    for g in ub.groups:
        assert all((p.pos_order, p.mom_degree, p.quad_n) == (g.key[0], g.key[2], g.key[3])
                   for p in (probs[i] for i in g.members))
        assert g.tet_offsets[0] == 0
        assert np.all(np.diff(g.tet_offsets) == [probs[i].nt for i in g.members])
        verts, tets, mu, refl, xyz, which = (x.numpy() for x in ub._concat(g))
        assert tets.shape[0] == g.tet_offsets[-1] and mu.shape[0] == tets.shape[0] and refl.shape[0] == tets.shape[0]
        boxes, voff, soff = [], 0, 0
        for m, i in enumerate(g.members):
            p = probs[i]
            nv, ns = p.verts.shape[0], len(p.source["xyz"])
            v = verts[voff:voff + nv]
            shift = v[0] - p.verts[0]
            # a pure translation, same connectivity shifted by the vertex offset
            assert np.allclose(v - shift, p.verts, atol=1e-12)
            assert np.array_equal(tets[g.tet_offsets[m]:g.tet_offsets[m + 1]], p.tets + voff)
            lo, hi = v.min(axis=0), v.max(axis=0)
            # the instance's sources, moved with it, lie on its own boundary
            pts = xyz[soff:soff + ns]
            assert np.allclose(pts - shift, p.source["xyz"], atol=1e-12)
            assert _on_box_surface(pts, lo, hi).all()
            assert np.array_equal(which[soff:soff + ns], np.arange(ns))
            boxes.append((lo, hi))
            voff += nv
            soff += ns
        # no two instances of a group overlap (nor touch)
        for a in range(len(boxes)):
            for b in range(a + 1, len(boxes)):
                sep = np.any((boxes[a][1] < boxes[b][0]) | (boxes[b][1] < boxes[a][0]))
                assert sep, f"instances {a} and {b} of group {g.key} overlap"
