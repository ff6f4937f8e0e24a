"""Pins of the stationary solve and the sources (paper Sec. 2, Eq. NSum / GovIE; Sec. 4)."""
import math

import numpy as np
import pytest

import synth
from oracle import assemble as oa
from oracle import basis as ob
from oracle import mesh as om
from oracle import quadrature as oq
from oracle import solve as osv
from oracle import sources as osrc


@pytest.fixture(scope="module")
def cube():
    p = synth.problem_c1()
    m = om.build_mesh(p.verts, p.tets, p.refl)
    bs = oa.Basis(p.pos_order, ob.LEGENDRE, p.mom_degree, p.quad_n, oq.SEAM_RULE)
    B, dest = oa.assemble(m, bs, p.mu)
    rho0 = osrc.project(m, bs, p.source)[0]
    return p, m, bs, B, dest, rho0


def mass_vector(m, bs):
    """m_J = int b_p psi_k ds dp (the density's total mass is m . rho)."""
    G = ob.gram(bs.mom_degree, bs.mom_family)
    v = np.zeros((4 * m.nt, bs.P, bs.M))
    v[:, 0, :] = np.sqrt(m.area.reshape(-1))[:, None] * G[:, 0][None, :]
    return v.ravel()


def test_neumann_direct_gmres_agree(cube):
    p, m, bs, B, dest, rho0 = cube
    A = osv.to_sparse(B, dest)
    r_lu = osv.solve_direct(A, rho0)
    r_nm, it, res = osv.neumann(A, rho0, tol=1e-12)
    r_gm, info = osv.gmres(A, rho0, tol=1e-13)
    assert res <= 1e-12 and it > 10
    assert osv.relres(A, rho0, r_lu) < 1e-14
    sc = np.abs(r_lu).max()
    assert np.abs(r_nm - r_lu).max() < 1e-10 * sc
    assert np.abs(r_gm - r_lu).max() < 1e-10 * sc


def test_block_apply_matches_sparse(cube):
    p, m, bs, B, dest, rho0 = cube
    A = osv.to_sparse(B, dest)
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    assert np.allclose(osv.apply(B, dest, x), A @ x, rtol=0, atol=1e-13)


def test_energy_balance_injected_equals_absorbed(cube):
    """mu = 0 and reflecting walls: in the stationary state all injected density
    leaves through the absorbing face x = 1 (Sec. 2, conservation of B)."""
    p, m, bs, B, dest, rho0 = cube
    A = osv.to_sparse(B, dest)
    rho = osv.solve_direct(A, rho0)
    full = synth.Problem(**{**p.__dict__, "refl": np.ones_like(p.refl)})
    m_full = om.build_mesh(full.verts, full.tets, full.refl)
    Bf, _ = oa.assemble(m_full, bs, full.mu)
    mv = mass_vector(m, bs)
    absorbed_slots = [4 * j + l for j in range(m.nt) for l in range(4) if m.nbr[j, l] < 0 and m.refl[j, l] == 0.0]
    y = osv.apply(Bf, dest, rho).reshape(4 * m.nt, bs.K)
    absorbed = sum(mv.reshape(4 * m.nt, -1)[s] @ y[s] for s in absorbed_slots)
    injected = mv @ rho0
    assert injected == pytest.approx(1.0, abs=1e-12)
    # per-bounce conservation holds to the n = 8 quadrature accuracy; ~300 bounces
    assert absorbed == pytest.approx(injected, rel=1e-4)


def test_face_flux_source_is_exact_in_legendre_basis():
    """cos(theta) = (psi_00 + psi_10/sqrt(3))/2, so the projection is exact."""
    ang = osrc.project_angular(lambda u, phi: u, 4, ob.LEGENDRE)
    ref = np.zeros(15)
    ref[0], ref[1] = 0.5, 0.5 / math.sqrt(3)
    assert np.abs(ang - ref).max() < 1e-13


@pytest.mark.parametrize("family", [ob.LEGENDRE, ob.ZERNIKE])
def test_sources_have_unit_flux(family):
    p = synth.problem_c2(n_cells=2)
    m = om.build_mesh(p.verts, p.tets, p.refl)
    bs = oa.Basis(1, family, 4, 4)
    mv = mass_vector(m, bs)
    g = osrc.project(m, bs, p.source)[0]
    assert mv @ g == pytest.approx(1.0, abs=1e-5)            # Gaussian tail beyond the face
    pts = synth.uniform_points_on_box_surface((1, 1, 1), 5, np.random.default_rng(0))
    r = osrc.project(m, bs, {"kind": "points", "xyz": pts})
    assert np.allclose(r @ mv, 1.0, atol=1e-13)


@pytest.mark.parametrize("family", [ob.LEGENDRE, ob.ZERNIKE])
def test_normal_incidence_source_pins(family):
    """Eq. RhoNeumann projected: G times the coefficients is the phi-average of the
    basis at the pole -- sqrt(2a+1) for b = 0 (Legendre), (-1)^(n/2) for m = 0
    (Zernike), zero otherwise -- and the projected density carries unit flux per
    area (checked by brute-force quadrature of the reconstructed function)."""
    D = 6
    ang = osrc.project_pole(D, family)
    G = ob.gram(D, family)
    ref = np.zeros(ang.size)
    for t in range(D + 1):
        for i in range(t + 1):
            k = t * (t + 1) // 2 + i
            if family == ob.LEGENDRE and i == 0:        # (a, b) = (t, 0)
                ref[k] = math.sqrt(2 * t + 1)
            if family == ob.ZERNIKE and t % 2 == 0 and -t + 2 * i == 0:
                ref[k] = (-1) ** (t // 2)
    assert np.abs(G @ ang - ref).max() < 1e-12
    xu, wu = np.polynomial.legendre.leggauss(40)
    xp, wp = np.polynomial.legendre.leggauss(40)
    U, PHI = np.meshgrid(0.5 * (xu + 1), np.pi * (xp + 1), indexing="ij")
    W = np.outer(0.5 * wu, np.pi * wp) * U
    f = ob.momentum(U.ravel(), PHI.ravel(), D, family) @ ang
    assert (W.ravel() @ f) == pytest.approx(1.0, abs=1e-12)
    # on a mesh: unit flux per area of the plane
    p = synth.problem_c1()
    m = om.build_mesh(p.verts, p.tets, p.refl)
    bs = oa.Basis(0, family, D, 4)
    r0 = osrc.project(m, bs, {"kind": "face_normal", "axis": 0, "value": 0.0, "flux": 1.0})[0]
    assert mass_vector(m, bs) @ r0 == pytest.approx(1.0, abs=1e-12)

