"""Pins of the receiver energy and the adjoint gradients (oracle/adjoint.py)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import adjoint as oj
from oracle import assemble as oa
from oracle import mesh as om
from oracle import quadrature as oq
from oracle import solve as osv
from oracle import sources as osrc


@pytest.mark.parametrize("i,m", [(0, 1), (1, 1), (0, 2), (2, 1), (1, 2), (0, 3)])
def test_moment_H_and_derivative(i, m):
    for a in (0.0, 1e-5, 3e-3, 0.02, 0.7, 3.0):
        ref = quad(lambda u: u ** i * (1 - u) ** m * (u if a == 0 else -math.expm1(-a * u) / a), 0, 1,
                   epsabs=1e-16, epsrel=1e-14)[0]
        assert oj.moment_H(i, m, a) == pytest.approx(ref, rel=1e-11)
        dref = quad(lambda u: u ** i * (1 - u) ** m * (-u * u / 2 if a == 0 else
                                                       (a * u * math.exp(-a * u) + math.expm1(-a * u)) / (a * a)),
                    0, 1, epsabs=1e-16, epsrel=1e-13)[0]
        assert oj.moment_dH(i, m, a) == pytest.approx(dref, rel=1e-8, abs=1e-14)


def test_energy_of_isotropic_radiance_is_four_pi_volume():
    """mu = 0, rho = 1 on every face (isotropic unit radiance): the chords from
    the four faces sweep the tet once per direction, so E = 4 pi V."""
    v = np.array([[0.1, 0.0, 0.0], [1.0, 0.2, 0.0], [0.3, 1.1, 0.1], [0.2, 0.3, 0.9]])
    m = om.build_mesh(v, np.array([[0, 1, 2, 3]]))
    for order in (0, 1):
        bs = oa.Basis(order, 0, 2, 16, oq.SEAM_RULE)
        g = oj.receiver_functional(m, bs, np.zeros(1), (-1, 2, -1, 2, -1, 2)).reshape(4, bs.P, bs.M)
        E = sum(math.sqrt(m.area[0, l]) * g[l, 0, 0] for l in range(4))
        assert E == pytest.approx(4 * math.pi * m.volume[0], rel=1e-10)


@pytest.fixture(scope="module")
def adj_problem():
    v, t = synth.kuhn_box((2, 1, 1), (1.0, 1.0, 1.0), 0.15, 3)
    refl = np.full((t.shape[0], 4), 0.8)
    mu = np.random.default_rng(1).uniform(0.1, 0.6, t.shape[0])
    bs = oa.Basis(1, 0, 2, 4, oq.SEAM_RULE)
    box = (0.5, 1.0, 0.0, 1.0, 0.0, 0.7)
    src = {"kind": "points", "xyz": synth.uniform_points_on_box_surface((1, 1, 1), 3, np.random.default_rng(2))}
    return v, t, refl, mu, bs, box, src


def _J(v, t, refl, mu, bs, box, rho0):
    m = om.build_mesh(v, t, refl)
    B, dest = oa.assemble(m, bs, mu)
    rho = osv.solve_direct(osv.to_sparse(B, dest), rho0)
    return oj.receiver_functional(m, bs, mu, box) @ rho


def test_adjoint_gradient_matches_central_differences(adj_problem):
    v, t, refl, mu, bs, box, src = adj_problem
    m = om.build_mesh(v, t, refl)
    w = np.array([0.7, 1.3, 0.4])
    rho0s = osrc.project(m, bs, src)
    rho0 = w @ rho0s
    B, dest = oa.assemble(m, bs, mu)
    A = osv.to_sparse(B, dest)
    rho = osv.solve_direct(A, rho0)
    g = oj.receiver_functional(m, bs, mu, box)
    lam = osv.solve_direct(A.T.tocsr(), g)
    dmu = oj.gradient_mu(m, bs, mu, lam, rho, box)
    dw = rho0s @ lam
    h = 1e-6
    for e in (0, 7, 10):
        mp, mm = mu.copy(), mu.copy()
        mp[e] += h
        mm[e] -= h
        fd = (_J(v, t, refl, mp, bs, box, rho0) - _J(v, t, refl, mm, bs, box, rho0)) / (2 * h)
        assert dmu[e] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(dmu).max())
    for s in range(3):
        wp, wm = w.copy(), w.copy()
        wp[s] += h
        wm[s] -= h
        fd = (_J(v, t, refl, mu, bs, box, wp @ rho0s) - _J(v, t, refl, mu, bs, box, wm @ rho0s)) / (2 * h)
        assert dw[s] == pytest.approx(fd, rel=1e-7)
    # duality: g . rho = lambda . rho0
    assert g @ rho == pytest.approx(lam @ rho0, rel=1e-12)
