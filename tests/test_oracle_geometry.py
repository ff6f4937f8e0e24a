"""Pins of the oracle's per-direction geometry (paper Sec. 3.3, the five steps).

Each check compares the oracle with something it does not compute itself:
exact polygon clipping, a derived closed form, a partition identity, or
numerical integration by scipy."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import geometry as og
from oracle import mesh as om
from oracle import quadrature as oq
from tests import refgeom as rg


@pytest.fixture(scope="module")
def jmesh():
    p = synth.problem_c2(n_cells=2)
    return om.build_mesh(p.verts, p.tets, p.refl)


def test_g_exp_series_matches_closed_form_and_limit():
    a = np.array([0.02, 0.05, 0.0999, 0.1, 0.3, 1.0, 3.0])
    ref = np.array([quad(lambda u: (1 - u) * math.exp(-x * u), 0, 1, epsabs=1e-15, epsrel=1e-15)[0] for x in a])
    assert np.allclose(og.g_exp(a), ref, rtol=1e-13, atol=0)
    assert og.g_exp(np.array([0.0]))[0] == 0.5          # mu = 0: the integral is the area


@pytest.mark.parametrize("i,m", [(0, 1), (0, 3), (1, 2), (2, 1), (2, 3)])
def test_moment_integral_matches_quadrature(i, m):
    for a in (0.0, 1e-4, 0.05, 0.7, 4.0):
        ref = quad(lambda u: u ** i * (1 - u) ** m * math.exp(-a * u), 0, 1, epsabs=1e-16, epsrel=1e-14)[0]
        assert og.moment_I(i, m, a) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("order", [0, 1])
def test_spatial_integral_matches_exact_clipping(jmesh, order):
    """Steps 1-3 (point O, L_max, analytic integral) equal the integral over the
    exactly clipped start set with a high-order triangle rule."""
    for (j, li, lo) in [(5, 0, 1), (5, 2, 3), (11, 3, 0), (30, 1, 2)]:
        d, _ = oq.block_nodes(jmesh, j, li, lo, 3, oq.PAPER_RULE)
        S = og.spatial_integrals(jmesh, j, li, lo, d, 0.7, order)
        for q in range(d.shape[0]):
            Sr = rg.clip_integral(jmesh.verts, jmesh.tets[j], li, lo, d[q], 0.7, order)
            assert np.abs(S[q] - Sr).max() <= 1e-13 * max(1.0, np.abs(Sr).max())


def test_start_sets_partition_the_inbound_face(jmesh):
    """For every direction the start sets of the three outbound faces tile ABC."""
    for (j, li) in [(0, 0), (7, 2), (40, 3)]:
        xg, wg = oq.gauss_legendre(5)
        z = jmesh.frame[j, li, 2]
        for patch, _ in oq.seven_pieces(jmesh, j, li):
            d, _ = oq.patch_nodes(patch, xg, wg, z)
            tot = sum(og.block_geometry(jmesh, j, li, lo, d)[1] for lo in range(4) if lo != li)
            assert np.allclose(tot, jmesh.area[j, li], rtol=1e-12)


def test_lmax_equals_three_volumes_over_silhouette(jmesh):
    """L_max from the paper's construction (ray from O) equals 3V/A_sil, A_sil the
    area of the tet's shadow perpendicular to d (projected-area argument)."""
    for (j, li) in [(2, 1), (9, 0), (33, 3)]:
        xg, wg = oq.gauss_legendre(4)
        z = jmesh.frame[j, li, 2]
        for patch, reach in oq.seven_pieces(jmesh, j, li):
            d, _ = oq.patch_nodes(patch, xg, wg, z)
            A_sil = sum(np.maximum(jmesh.area[j, g] * (d @ jmesh.n_out[j, g]), 0.0) for g in range(4) if g != li)
            for lo in reach:
                _, area, Lmax, _ = og.block_geometry(jmesh, j, li, lo, d)
                assert np.allclose(Lmax, 3 * jmesh.volume[j] / A_sil, rtol=1e-11)


def test_regions_reach_exactly_their_faces(jmesh):
    """Inside region r the start set of face F is non-empty iff F is listed for r."""
    for (j, li) in [(1, 2), (17, 0)]:
        xg, wg = oq.gauss_legendre(4)
        z = jmesh.frame[j, li, 2]
        for patch, reach in oq.seven_pieces(jmesh, j, li):
            d, _ = oq.patch_nodes(patch, xg, wg, z)
            for lo in range(4):
                if lo == li:
                    continue
                area = og.block_geometry(jmesh, j, li, lo, d)[1]
                if lo in reach:
                    assert np.all(area > 0)
                else:
                    assert np.all(area == 0)
