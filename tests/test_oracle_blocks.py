"""Physics pins of whole blocks of B (paper Sec. 2 and Sec. 3.2).

* regular tetrahedron view factors (symmetry, golden file);
* reciprocity of straight-ray transport (time reversal of a chord);
* conservation with w = 1 (Sec. 2: the operator then preserves the density);
* Monte Carlo ray tracing of whole blocks on one tetrahedron.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import assemble as oa
from oracle import basis as ob
from oracle import mesh as om
from oracle import quadrature as oq
from tests import refgeom as rg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def regular_tet():
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) * 0.5
    return om.build_mesh(v, np.array([[0, 1, 2, 3]]))


@pytest.fixture(scope="module")
def jmesh():
    p = synth.problem_c2(n_cells=2)
    return om.build_mesh(p.verts, p.tets, p.refl)


@pytest.mark.parametrize("family", [ob.LEGENDRE, ob.ZERNIKE])
def test_regular_tet_view_factor(family):
    g = _golden("regular_tet.txt")
    m = regular_tet()
    bs = oa.Basis(0, family, 2, 16, oq.PAPER_RULE)
    for li in range(4):
        for lo in range(4):
            if lo != li:
                T, _, _ = oa.block_T(m, bs, 0.0, 0, li, lo)
                assert T[0, 0] == pytest.approx(g["t00"], abs=1e-10)


@pytest.mark.parametrize("order", [0, 1])
def test_reciprocity(jmesh, order):
    """A chord traversed backwards: for theta-only modes (b = 0) and either
    position order, T(i -> j)[(p',a'),(p,a)] = T(j -> i)[(p,a),(p',a')], with or
    without damping (exp(-mu L) is symmetric in the chord)."""
    D = 4
    idx = ob.momentum_index(D, ob.LEGENDRE)
    sel = [k for k, (a, b) in enumerate(idx) if b == 0]
    P, M = (1, len(idx)) if order == 0 else (3, len(idx))
    rows = [p * M + k for p in range(P) for k in sel]
    bs = oa.Basis(order, ob.LEGENDRE, D, 24, oq.SEAM_RULE)
    for j in (0, 13):
        for (fi, fj) in ((0, 1), (2, 3), (1, 3)):
            Tij, _, _ = oa.block_T(jmesh, bs, 0.4, j, fi, fj)
            Tji, _, _ = oa.block_T(jmesh, bs, 0.4, j, fj, fi)
            A = Tij[np.ix_(rows, rows)]
            B = Tji[np.ix_(rows, rows)].T
            assert np.abs(A - B).max() <= 1e-7 * np.abs(A).max()


@pytest.mark.parametrize("family,rule,tol", [(ob.ZERNIKE, oq.PAPER_RULE, 1e-9), (ob.LEGENDRE, oq.SEAM_RULE, 1e-9),
                                             (ob.LEGENDRE, oq.PAPER_RULE, 5e-2)])
def test_conservation_without_losses(jmesh, family, rule, tol):
    """mu = 0, w = 1: the density leaving a tet equals the density entering it,
    sum_F sqrt|F| T_F[(0,0),(p,k)] = sqrt|F_in| delta_p0 int psi_k cos dOmega.
    Tight for smooth integrands (Zernike, or Legendre on the seam rule); the
    paper's seven regions with the Legendre basis integrate the phi-seam badly."""
    D = 6
    n = 32 if rule == oq.PAPER_RULE else 24
    bs = oa.Basis(1, family, D, n, rule)
    G = ob.gram(D, family)
    M = bs.M
    for (j, li) in [(5, 0), (22, 3)]:
        tot = np.zeros(bs.K)
        for lo in range(4):
            if lo != li:
                T, _, _ = oa.block_T(jmesh, bs, 0.0, j, li, lo)
                tot += math.sqrt(jmesh.area[j, lo]) * T[0]
        ref = np.zeros(bs.K)
        ref[:M] = math.sqrt(jmesh.area[j, li]) * G[:, 0]
        assert np.abs(tot - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("order,mu", [(0, 0.0), (1, 0.8)])
def test_block_matches_monte_carlo(jmesh, order, mu):
    """Whole unnormalised blocks vs Monte Carlo ray tracing (independent tracer,
    frames and bases restated in tests/refgeom.py), within 5 standard errors."""
    rng = np.random.default_rng(1234 + order)
    D = 3
    bs = oa.Basis(order, ob.LEGENDRE, D, 24, oq.SEAM_RULE)
    for (j, li, lo) in [(6, 1, 2), (40, 3, 0)]:
        T, slot, _ = oa.block_T(jmesh, bs, mu, j, li, lo)
        tr = jmesh.nbr[j, lo] >= 0
        dest = rg.face_frame(jmesh.verts, jmesh.tets[slot // 4], slot % 4)
        X, se = rg.mc_block(jmesh.verts, jmesh.tets[j], li, lo, mu, D, order, 1_500_000, rng,
                            dest_frame=dest, reflect=not tr)
        z = np.abs(T - X) / np.maximum(se, 1e-6 * np.abs(T).max())
        assert z.max() < 5.5
