"""The seeded synthetic inputs follow the stated recipe (sizes, fields, sources).

They hold no arithmetic of the method; these checks keep the workloads the
benches and tests run on what the design notes describe."""
import math

import numpy as np
import pytest

import synth


def volumes(verts, tets):
    a, b, c, d = (verts[tets[:, i]] for i in range(4))
    return np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a) / 6.0


def on_box_surface(pts, size, tol=1e-12):
    s = np.asarray(size)
    near = (np.abs(pts) <= tol) | (np.abs(pts - s) <= tol)
    inside = np.all((pts >= -tol) & (pts <= s + tol), axis=1)
    return inside & near.any(axis=1)


@pytest.mark.parametrize("cells,size,jitter", [((1, 1, 1), (1.0, 1.0, 1.0), 0.0), ((3, 2, 4), (2.0, 1.0, 1.5), 0.2)])
def test_kuhn_box_fills_the_box_with_conforming_tets(cells, size, jitter):
    """6 tets per cell, all positively oriented, volumes summing to the box; every
    face is shared by two tets or lies on a box plane."""
    v, t = synth.kuhn_box(cells, size, jitter=jitter, seed=3)
    assert t.shape[0] == 6 * math.prod(cells)
    vol = np.abs(volumes(v, t))
    assert vol.min() > 0 and vol.sum() == pytest.approx(math.prod(size), rel=1e-12)
    faces = np.sort(synth.face_vertices(t).reshape(-1, 3), axis=1)
    keys, counts = np.unique(faces, axis=0, return_counts=True)
    assert counts.max() == 2
    for f in keys[counts == 1]:
        assert np.any([np.all(np.abs(v[f, ax] - val) < 1e-12) for ax in range(3) for val in (0.0, size[ax])])


def test_points_are_uniform_by_area_on_the_box_surface():
    size = (2.0, 1.0, 3.0)
    pts = synth.uniform_points_on_box_surface(size, 60000, np.random.default_rng(0))
    assert on_box_surface(pts, size).all()
    areas = np.array([size[1] * size[2], size[0] * size[2], size[0] * size[1]]) * 2
    frac = np.array([np.mean((np.abs(pts[:, ax]) < 1e-12) | (np.abs(pts[:, ax] - size[ax]) < 1e-12))
                     for ax in range(3)])
    assert np.abs(frac - areas / areas.sum()).max() < 0.01


def test_box8_recipe():
    p = synth.problem_c2()
    assert p.nt == 3072 and (p.pos_order, p.mom_degree, p.quad_n) == (1, 8, 12)
    assert np.all(p.mu == 0.05) and np.all(p.refl == 0.9)
    assert p.source["kind"] == "gauss_patch" and p.source["sigma"] == 0.1


def test_box32_recipe():
    p = synth.problem_c3()
    assert p.nt == 49152 and (p.pos_order, p.mom_degree, p.quad_n) == (0, 12, 16)
    lm = np.log(p.mu)
    assert lm.mean() == pytest.approx(math.log(0.02), abs=0.01) and lm.std() == pytest.approx(0.5, abs=0.01)
    pts = p.source["xyz"]
    assert pts.shape == (128, 3) and on_box_surface(pts, (2.0, 1.0, 1.0)).all()
    assert np.abs(volumes(p.verts, p.tets)).sum() == pytest.approx(2.0, rel=1e-12)


def test_uneven_batch_recipe():
    probs = synth.problem_c5()
    assert len(probs) == 256
    assert sum(p.nt for p in probs) == 1439370
    assert {p.mom_degree for p in probs} == {4, 6, 8, 10}
    for p in probs:
        assert p.quad_n == p.mom_degree + 4 and p.pos_order == 0
        assert np.all(p.mu == p.mu[0]) and 0.0 <= p.mu[0] <= 0.1
        assert p.size[0] == 1.0 and 1.0 <= p.size[1] <= 4.0 and 1.0 <= p.size[2] <= 4.0
        assert p.source["xyz"].shape == (4, 3) and on_box_surface(p.source["xyz"], p.size).all()
    nts = np.array([p.nt for p in probs])
    assert (nts.min(), nts.max()) == (384, 20412)   # target log-uniform in [500, 20000], cells rounded
