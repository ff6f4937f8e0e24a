"""Pins of the oracle's basis functions (paper Sec. 3.1)."""
import math
import os

import numpy as np
import pytest

from oracle import basis as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _product_rule(nu=40, nphi=80):
    """Product Gauss rule on the hemisphere in (u = cos theta, phi), weight u du dphi."""
    xu, wu = np.polynomial.legendre.leggauss(nu)
    xp, wp = np.polynomial.legendre.leggauss(nphi)
    u, phi = 0.5 * (xu + 1), np.pi * (xp + 1)
    U, PHI = np.meshgrid(u, phi, indexing="ij")
    return U.ravel(), PHI.ravel(), (np.outer(0.5 * wu, np.pi * wp) * U).ravel()


@pytest.mark.parametrize("D", [0, 1, 4, 8, 12])
def test_legendre_gram_closed_form(D):
    """The closed-form Gram matrix equals brute-force integration of psi psi^T
    cos(theta) dOmega (a product Gauss rule exact for these polynomials)."""
    u, phi, w = _product_rule()
    psi = ob.legendre_momentum(u, phi, D)
    G = (psi * w[:, None]).T @ psi
    assert np.abs(G - ob.gram(D, ob.LEGENDRE)).max() < 1e-12


def test_zernike_recurrence_matches_explicit_table():
    rho = np.linspace(0, 1, 11)
    with open(os.path.join(GOLDEN, "zernike_radial.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            vals = [int(v) for v in line.split()]
            n, m, coef = vals[0], vals[1], vals[2:]
            ref = sum(c * rho ** (n - 2 * i) for i, c in enumerate(coef))
            assert np.allclose(ob.zernike_radial(n, m, rho), ref, atol=1e-13)


def test_zernike_recurrence_matches_factorial_formula():
    rho = np.linspace(0, 1, 7)
    for n in range(13):
        for m in range(n % 2, n + 1, 2):
            ref = sum((-1) ** k * math.factorial(n - k)
                      / (math.factorial(k) * math.factorial((n + m) // 2 - k) * math.factorial((n - m) // 2 - k))
                      * rho ** (n - 2 * k) for k in range((n - m) // 2 + 1))
            assert np.allclose(ob.zernike_radial(n, m, rho), ref, atol=1e-10)


@pytest.mark.parametrize("D", [4, 10])
def test_zernike_orthogonality(D):
    """int Z Z' rho drho dphi = eps pi/(2n+2) delta delta (Sec. 3.1); the same
    integral is cos(theta) dOmega on the hemisphere."""
    xr, wr = np.polynomial.legendre.leggauss(30)
    r = 0.5 * (xr + 1)
    phi = 2 * np.pi * np.arange(64) / 64
    R, PHI = np.meshgrid(r, phi, indexing="ij")
    W = np.outer(0.5 * wr * r, np.full(64, 2 * np.pi / 64)).ravel()
    cos_t = np.sqrt(1 - R.ravel() ** 2)
    Z = ob.zernike_momentum(cos_t, PHI.ravel(), D)
    G = (Z * W[:, None]).T @ Z
    assert np.abs(G - ob.gram(D, ob.ZERNIKE)).max() < 1e-12


def test_zernike_pole_values():
    """Z_n^0 = (-1)^(n/2) and Z_n^m = 0 (m != 0) at theta = 0 (Sec. 3.4)."""
    Z = ob.zernike_momentum(np.array([1.0]), np.array([0.7]), 10)[0]
    for k, (n, m) in enumerate(ob.momentum_index(10, ob.ZERNIKE)):
        assert Z[k] == pytest.approx((-1) ** (n // 2) if m == 0 else 0.0, abs=1e-14)


def test_p1_position_basis_orthonormal():
    x, w = np.polynomial.legendre.leggauss(8)
    u, wu = 0.5 * (x + 1), 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    W = (np.outer(wu, wu) * (1 - U)).ravel()
    l1 = U.ravel()
    l2 = (V * (1 - U)).ravel()
    lam = np.stack([1 - l1 - l2, l1, l2], axis=1)
    for area in (0.3, 2.0):
        b = ob.position_basis(lam, area, 1)
        G = (b * (2 * area * W)[:, None]).T @ b
        assert np.abs(G - np.eye(3)).max() < 1e-13


def test_direction_angles():
    fr = np.eye(3)
    d = np.array([[0, 0, 1.0], [1 / math.sqrt(2), 1 / math.sqrt(2), 0], [0.6, -0.8 * 0.6, 0.8 * 0.8],
                  [1.0, 1e-16, 0.0]])
    c, phi = ob.direction_angles(d, fr)
    assert c[0] == 1.0 and phi[1] == pytest.approx(math.pi / 4)
    assert phi[2] == pytest.approx(2 * math.pi + math.atan2(-0.48, 0.6))
    assert phi[3] == 0.0
