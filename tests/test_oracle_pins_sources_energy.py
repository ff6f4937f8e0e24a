"""Independent pins of two oracle parts that the other pins reach only in part:

* the receiver energy at mu > 0 (oracle/adjoint.py, Sec. 4.1 Eq. IntDens
  integrated over a tet), against a Monte Carlo chord tracer that scores
  (1 - exp(-mu L)) / mu along each sampled ray (tests/refgeom.py);
* the position moments of the Gaussian-patch source for the linear position
  basis (oracle/sources.py), against an independent triangle rule on a
  subdivided face (tests/refgeom.py), and their limits: a flat patch gives
  zero linear moments, and the moments of a wide patch approach the affine
  closed form of its Taylor expansion.

Each pin is shown to fail when a plausible mistake is planted in the oracle:
L exp(-mu L) scored instead of (1 - exp(-mu L))/mu, and the linear position
functions evaluated with cyclically shifted barycentric coordinates.
"""
import math

import numpy as np
import pytest

import synth
from oracle import adjoint as oj
from oracle import assemble as oa
from oracle import basis as ob
from oracle import geometry as og
from oracle import mesh as om
from oracle import quadrature as oq
from oracle import sources as osrc
from tests import refgeom as rg

MC_Z = 5.0          # Monte Carlo bound, in standard errors
MOMENT_REL = 1e-10  # Gaussian-patch moments vs the independent rule

TET = np.array([[0.1, 0.0, 0.0], [1.0, 0.2, 0.0], [0.3, 1.1, 0.1], [0.2, 0.3, 0.9]])


def energy_z(mu, order, D=2, nsamp=1_500_000, seed=11):
    """Largest |g - MC| over faces, position and momentum functions, in standard errors."""
    m = om.build_mesh(TET, np.array([[0, 1, 2, 3]]))
    bs = oa.Basis(order, ob.LEGENDRE, D, 16, oq.SEAM_RULE)
    g = oj.receiver_functional(m, bs, np.array([mu]), (-1, 2, -1, 2, -1, 2)).reshape(4, bs.P, bs.M)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for l in range(4):
        mean, se = rg.mc_energy(TET, np.array([0, 1, 2, 3]), l, mu, D, order, nsamp, rng)
        worst = max(worst, float((np.abs(g[l] - mean) / np.maximum(se, 1e-12)).max()))
    return worst


@pytest.mark.parametrize("mu,order", [(0.3, 0), (1.5, 0), (4.0, 1)])
def test_receiver_energy_matches_monte_carlo_chords(mu, order):
    assert energy_z(mu, order) < MC_Z


def test_receiver_energy_planted_chord_weight_is_caught(monkeypatch):
    # L exp(-mu L) in place of (1 - exp(-mu L))/mu: H_{i,m} replaced by I_{i+1,m};
    # both agree at mu = 0, so the mu = 0 energy pin cannot see it
    monkeypatch.setattr(oj, "moment_H", lambda i, m, a: og.moment_I(i + 1, m, a))
    assert energy_z(1.5, 0) > 4 * MC_Z


def _patch_moments_case(sigma=0.1, center=(0.0, 0.5, 0.5)):
    p = synth.problem_c2(n_cells=4)
    m = om.build_mesh(p.verts, p.tets, p.refl)
    bs = oa.Basis(1, ob.LEGENDRE, 2, 4, oq.PAPER_RULE)
    rho0 = osrc.project(m, bs, {"kind": "gauss_patch", "axis": 0, "value": 0.0, "center": center,
                                "sigma": sigma, "flux": 1.0})[0].reshape(4 * m.nt, bs.P, bs.M)
    slots = [s for s in range(4 * m.nt) if m.nbr[s // 4, s % 4] < 0
             and np.all(p.verts[rg.face_ids(p.tets[s // 4], s % 4)][:, 0] == 0.0)]
    return p, m, bs, rho0, slots


def patch_moment_error(sigma=0.1, center=(0.0, 0.5, 0.5)):
    """Largest relative gap between the oracle's position moments and the
    independent rule, over every face of the source plane.  The oracle's
    coefficients are flux * mom[p] * ang[k]; the momentum factor is divided out
    with the momentum function of largest weight."""
    p, m, bs, rho0, slots = _patch_moments_case(sigma, center)
    k = int(np.argmax(np.abs(rho0[slots].sum(axis=(0, 1)))))
    ref = np.array([rg.gauss_patch_moments(p.verts, rg.face_ids(p.tets[s // 4], s % 4), center, sigma, 1)
                    for s in slots])
    got = np.array([rho0[s, :, k] for s in slots])
    ang = got[:, 0].sum() / ref[:, 0].sum()          # the common momentum factor
    return float(np.abs(got / ang - ref).max() / np.abs(ref).max())


def test_gauss_patch_linear_moments_match_independent_rule():
    assert patch_moment_error() < MOMENT_REL


def test_gauss_patch_linear_moments_vanish_for_a_flat_patch():
    """sigma -> infinity: the density is constant on every face, and the two
    linear functions have zero mean (they are orthogonal to the constant)."""
    p, m, bs, rho0, slots = _patch_moments_case(sigma=1e4)
    lin = np.abs(np.array([rho0[s, 1:, :] for s in slots])).max()
    const = np.abs(np.array([rho0[s, 0, :] for s in slots])).max()
    assert lin < 1e-9 * const


def _tri_monomial(e, A):
    """int over a triangle of area A of l0^e0 l1^e1 l2^e2 = 2 A e0! e1! e2! / (e0+e1+e2+2)!."""
    return 2.0 * A * math.prod(math.factorial(k) for k in e) / math.factorial(sum(e) + 2)


def test_gauss_patch_moments_of_a_wide_patch_follow_the_quadratic_closed_form():
    """For sigma much larger than the box, exp(-r^2/(2 s^2)) = 1 - r^2/(2 s^2) +
    O(r^4/s^4) with r^2 = |sum_i l_i (V_i - c)|^2 quadratic in the barycentrics,
    so every position moment is a sum of exact barycentric monomial integrals."""
    sigma, c = 20.0, np.array([0.0, 0.1, 0.2])
    p, m, bs, rho0, slots = _patch_moments_case(sigma=sigma, center=tuple(c))
    k = int(np.argmax(np.abs(rho0[slots].sum(axis=(0, 1)))))
    got_all, ref_all = [], []
    for s in slots:
        ids = rg.face_ids(p.tets[s // 4], s % 4)
        V = p.verts[ids]
        A = 0.5 * np.linalg.norm(np.cross(V[1] - V[0], V[2] - V[0]))
        Gm = (V - c) @ (V - c).T                      # r^2 = l^T Gm l
        # integrals of l_a * 1 and l_a * l_i * l_j over the face
        e1 = [_tri_monomial(tuple(int(t == a) for t in range(3)), A) for a in range(3)]
        q = [sum(Gm[i, j] * _tri_monomial(tuple(int(t == a) + int(t == i) + int(t == j) for t in range(3)), A)
                 for i in range(3) for j in range(3)) for a in range(3)]
        norm = 1.0 / (2 * math.pi * sigma ** 2)
        mom_l = [norm * (e1[a] - q[a] / (2 * sigma ** 2)) for a in range(3)]   # int l_a f
        mom_1 = sum(mom_l)                                                    # int f (sum l_a = 1)
        ref = np.array([mom_1 / math.sqrt(A), math.sqrt(6 / A) * (mom_l[1] - mom_l[0]),
                        math.sqrt(2 / A) * (3 * mom_l[2] - mom_1)])
        got_all.append(rho0[s, :, k])
        ref_all.append(ref)
    got, ref = np.array(got_all), np.array(ref_all)
    ang = got[:, 0].sum() / ref[:, 0].sum()
    lin = np.abs(ref[:, 1:]).max()
    # the next term of the expansion is r^4/(8 s^4): below 1e-2 of the r^2 term here
    assert np.abs(got[:, 1:] / ang - ref[:, 1:]).max() < 1e-2 * lin


def test_gauss_patch_planted_barycentric_shift_is_caught(monkeypatch):
    _pb = ob.position_basis
    monkeypatch.setattr(ob, "position_basis", lambda lam, area, order: _pb(lam[..., [2, 0, 1]], area, order))
    assert patch_moment_error() > 1e6 * MOMENT_REL
