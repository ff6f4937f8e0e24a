"""Basis functions of the product expansion (paper Sec. 3.1, Eq. FBApprox).

Position: orthonormal on each face.  The paper uses the piecewise constant
b = 1/sqrt(|face|) and mentions higher order position bases as an option
(Sec. 4.1, last paragraph); order 1 here is the orthonormal linear basis
    e0 = 1/sqrt(A), e1 = sqrt(6/A) (l1 - l0), e2 = sqrt(2/A) (3 l2 - 1)
in the barycentric coordinates l0, l1, l2 of the face's vertices taken in
increasing global id.

Momentum (direction) on the inward hemisphere, total degree <= D, two families:
  * family 0 ("legendre"): psi_(a,b) = p_a(2 cos(theta) - 1) p_b(phi/pi - 1),
    p_a = sqrt(2a+1) P_a, ordered by t = a+b = 0..D, then b = 0..t;
  * family 1 ("zernike", the paper's basis, Sec. 3.1): Z_n^m(sin(theta), phi),
    ordered by n = 0..D, then m = -n, -n+2, ..., n.

The Galerkin inner product is the one of Eq. Bapprox: ds dp with p the
tangential momentum, i.e. dp = rho d(rho) d(phi) = cos(theta) dOmega on the
hemisphere (the "flux measure").  Zernike polynomials are orthogonal under it
(Sec. 3.1); the Legendre family is not, so its Gram matrix is returned too.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre

LEGENDRE = 0
ZERNIKE = 1

# A direction whose frame-y component is this small (relative to a unit vector)
# is taken to lie on the half-plane phi = 0 (x > 0).
SEAM_SNAP = 1e-13


def momentum_count(D):
    return (D + 1) * (D + 2) // 2


def momentum_index(D, family):
    if family == LEGENDRE:
        return [(t - b, b) for t in range(D + 1) for b in range(t + 1)]
    return [(n, m) for n in range(D + 1) for m in range(-n, n + 1, 2)]


def direction_angles(d, frame):
    """cos(theta) and phi in [0, 2 pi) of unit directions d [Q,3] in a face frame (rows x,y,z).

    Eq. sphpol: theta = arccos(g3), phi = arctan(f2/f1) mod 2 pi, read as the
    two-argument arctangent."""
    dx = d @ frame[0]
    dy = d @ frame[1]
    dz = d @ frame[2]
    phi = np.arctan2(dy, dx)
    phi = np.where(phi < 0.0, phi + 2.0 * np.pi, phi)
    phi = np.where((np.abs(dy) <= SEAM_SNAP) & (dx > 0.0), 0.0, phi)
    return dz, phi


def legendre_momentum(cos_t, phi, D):
    x = 2.0 * cos_t - 1.0
    y = phi / np.pi - 1.0
    px = [math.sqrt(2 * a + 1) * eval_legendre(a, x) for a in range(D + 1)]
    py = [math.sqrt(2 * b + 1) * eval_legendre(b, y) for b in range(D + 1)]
    return np.stack([px[a] * py[b] for (a, b) in momentum_index(D, LEGENDRE)], axis=-1)


def zernike_radial(n, m, rho):
    """R_n^m by the three-term recurrence of Sec. 3.1 (R_0^0 = 1, R_1^1 = rho;
    R_n^m = 0 when m > n or n - m is odd)."""
    m = abs(m)
    if m > n or (n - m) % 2:
        return np.zeros_like(rho)
    if n == 0:
        return np.ones_like(rho)
    if n == 1:
        return np.array(rho, dtype=np.float64, copy=True)
    return rho * (zernike_radial(n - 1, abs(m - 1), rho) + zernike_radial(n - 1, m + 1, rho)) \
        - zernike_radial(n - 2, m, rho)


def zernike_momentum(cos_t, phi, D):
    rho = np.sqrt(np.clip(1.0 - cos_t * cos_t, 0.0, None))    # rho = sin(theta)
    cols = []
    for (n, m) in momentum_index(D, ZERNIKE):
        r = zernike_radial(n, m, rho)
        cols.append(r * (np.cos(m * phi) if m >= 0 else np.sin(-m * phi)))
    return np.stack(cols, axis=-1)


def momentum(cos_t, phi, D, family):
    if family == LEGENDRE:
        return legendre_momentum(cos_t, phi, D)
    return zernike_momentum(cos_t, phi, D)


def gram(D, family):
    """Gram matrix of the momentum family under cos(theta) dOmega on the hemisphere.

    Zernike: diag(eps_m pi / (2n + 2)) with eps_0 = 2, else 1 (Sec. 3.1).
    Legendre: with u = cos(theta), x = 2u - 1, y = phi/pi - 1 the measure is
    u du dphi = (pi/4)(1 + x) dx dy, so the (a,b),(a',b') entry is
    (pi/4) * int (1+x) p_a p_a' dx * int p_b p_b' dy
      = pi * [delta_aa' + J_aa'] * delta_bb',
    with J the Jacobi matrix of x in the orthonormal Legendre basis,
    J_(a,a+1) = (a+1)/sqrt((2a+1)(2a+3)).
    """
    idx = momentum_index(D, family)
    K = len(idx)
    G = np.zeros((K, K))
    if family == ZERNIKE:
        for i, (n, m) in enumerate(idx):
            G[i, i] = (2.0 if m == 0 else 1.0) * np.pi / (2 * n + 2)
        return G
    pos = {ab: i for i, ab in enumerate(idx)}
    for i, (a, b) in enumerate(idx):
        G[i, i] = np.pi
        if (a + 1, b) in pos:
            j = pos[(a + 1, b)]
            G[i, j] = G[j, i] = np.pi * (a + 1) / math.sqrt((2 * a + 1) * (2 * a + 3))
    return G


def position_count(order):
    return 1 if order == 0 else 3


def position_basis(lam, area, order):
    """Orthonormal position basis on a face at barycentric coordinates lam [...,3]
    (w.r.t. the face's vertices in increasing global id)."""
    lam = np.asarray(lam, dtype=np.float64)
    e0 = np.full(lam.shape[:-1], 1.0 / math.sqrt(area))
    if order == 0:
        return e0[..., None]
    e1 = math.sqrt(6.0 / area) * (lam[..., 1] - lam[..., 0])
    e2 = math.sqrt(2.0 / area) * (3.0 * lam[..., 2] - 1.0)
    return np.stack([e0, e1, e2], axis=-1)
