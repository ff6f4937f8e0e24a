"""Pins of the oracle's direction quadrature (paper Sec. 3.4)."""
import numpy as np
import pytest

import synth
from oracle import assemble as oa
from oracle import geometry as og
from oracle import mesh as om
from oracle import quadrature as oq


@pytest.fixture(scope="module")
def jmesh():
    p = synth.problem_c2(n_cells=2)
    return om.build_mesh(p.verts, p.tets, p.refl)


@pytest.mark.parametrize("n", [1, 4, 8, 12, 16])
def test_gauss_legendre_exact_on_monomials(n):
    x, w = oq.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert (w * x ** k).sum() == pytest.approx(exact, abs=1e-14)


@pytest.mark.parametrize("j,l_in", [(0, 0), (3, 1), (21, 2), (47, 3)])
def test_seven_regions_cover_hemisphere_flux_measure(jmesh, j, l_in):
    """sum over the seven regions of int cos(theta) dOmega = pi, spectrally in n."""
    z = jmesh.frame[j, l_in, 2]
    errs = []
    for n in (4, 8, 16, 32):
        xg, wg = oq.gauss_legendre(n)
        tot = sum(oq.patch_nodes(p, xg, wg, z)[1].sum() for p, _ in oq.seven_pieces(jmesh, j, l_in))
        errs.append(abs(tot - np.pi))
    assert errs[-1] < 1e-12
    assert errs[0] > errs[1] > errs[2] > errs[3]


def test_cube_regions_cover_hemisphere():
    p = synth.problem_c1()
    m = om.build_mesh(p.verts, p.tets, p.refl)
    xg, wg = oq.gauss_legendre(20)
    for j in range(6):
        for l in range(4):
            tot = sum(oq.patch_nodes(pc, xg, wg, m.frame[j, l, 2])[1].sum() for pc, _ in oq.seven_pieces(m, j, l))
            assert tot == pytest.approx(np.pi, abs=1e-12)


@pytest.mark.parametrize("rule", [oq.PAPER_RULE, oq.SEAM_RULE])
def test_block_cells_tile_the_reachable_set(jmesh, rule):
    """sum_F int_{cells of F} omega_F cos(theta) dOmega = pi, omega_F the fraction of
    the inbound face whose rays exit through F (the cells of each block must
    tile exactly the directions that reach F)."""
    for (j, li) in [(4, 0), (29, 3)]:
        tot = 0.0
        for lo in range(4):
            if lo == li:
                continue
            d, W = oq.block_nodes(jmesh, j, li, lo, 20, rule)
            area = og.block_geometry(jmesh, j, li, lo, d)[1]
            tot += (W * area).sum() / jmesh.area[j, li]
        assert tot == pytest.approx(np.pi, abs=1e-10)


def test_seam_rule_keeps_poles_at_cell_corners(jmesh):
    """Every seam-rule cell touching a pole has it as its collapsed corner, and no
    cell straddles a seam half-plane phi = 0 of the inbound or destination frame."""
    for (j, li, lo) in [(3, 0, 1), (11, 1, 0), (20, 3, 2)]:
        z_in = jmesh.frame[j, li, 2]
        n_f = jmesh.n_out[j, lo]
        slot = jmesh.nbr[j, lo]
        fd = jmesh.frame[slot // 4, slot % 4] if slot >= 0 else jmesh.frame[j, lo]
        for cell in oq.block_cells(jmesh, j, li, lo, oq.SEAM_RULE):
            xg, wg = oq.gauss_legendre(6)
            d, _ = oq.patch_nodes(cell, xg, wg, z_in)
            for fr in (jmesh.frame[j, li], fd):
                sy = d @ fr[1]
                sx = d @ fr[0]
                assert np.all(sy >= -1e-12) or np.all(sy <= 1e-12)
                assert np.all(sx >= -1e-12) or np.all(sx <= 1e-12)
            for pole in (z_in, n_f):
                dist = [np.linalg.norm(v - pole) for v in cell]
                if min(dist) < 1e-9:
                    assert dist[0] < 1e-12 and dist[3] < 1e-12


def test_seam_rule_converges_for_legendre_basis(jmesh):
    """Quadrature-order convergence: successive differences fall fast with n."""
    diffs = []
    prev = None
    for n in (8, 16, 32):
        B, _ = oa.block(jmesh, oa.Basis(0, 0, 6, n, oq.SEAM_RULE), 0.05, 3, 0, 1)
        if prev is not None:
            diffs.append(np.abs(B - prev).max() / np.abs(B).max())
        prev = B
    assert diffs[1] < 1e-5 and diffs[1] < 1e-3 * diffs[0]
