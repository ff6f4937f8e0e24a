"""Stationary density (paper Sec. 2, Eq. NSum and Eq. GovIE).

rho = sum_n B^n rho0 (Neumann series), equivalently (I - B) rho = rho0.
The relative residual ||rho0 - (I - B) rho|| / ||rho0|| is the stopping
measure; for the Neumann partial sum rho_n = sum_{k<=n} B^k rho0 it equals
||B^{n+1} rho0|| / ||rho0||.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def to_sparse(B, dest):
    """Global sparse matrix from blocks B[nt][4][3][K][K] and dest[nt][4]."""
    nt, _, _, K, _ = B.shape
    rows, cols, vals = [], [], []
    rr, cc = np.meshgrid(np.arange(K), np.arange(K), indexing="ij")
    for j in range(nt):
        for l_out in range(4):
            ins = [l for l in range(4) if l != l_out]
            for s, l_in in enumerate(ins):
                rows.append(dest[j, l_out] * K + rr.ravel())
                cols.append((4 * j + l_in) * K + cc.ravel())
                vals.append(B[j, l_out, s].ravel())
    n = 4 * nt * K
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def apply(B, dest, x):
    """y = B x for x [..., 4*nt*K] (block form, no sparse matrix)."""
    nt, _, _, K, _ = B.shape
    xs = x.reshape(x.shape[:-1] + (nt, 4, K))
    y = np.zeros_like(xs)
    for l_out in range(4):
        ins = [l for l in range(4) if l != l_out]
        acc = sum(np.einsum("jrc,...jc->...jr", B[:, l_out, s], xs[..., :, l_in, :])
                  for s, l_in in enumerate(ins))
        d = dest[:, l_out]
        y.reshape(x.shape[:-1] + (4 * nt, K))[..., d, :] = acc
    return y.reshape(x.shape)


def relres(A, rho0, rho):
    n = A.shape[0]
    r = rho0 - (rho - A @ rho)
    return np.linalg.norm(r) / np.linalg.norm(rho0)


def solve_direct(A, rho0):
    """(I - B) rho = rho0 by sparse LU."""
    n = A.shape[0]
    return spla.spsolve((sp.identity(n, format="csc") - A.tocsc()), rho0)


def neumann(A, rho0, tol=1e-12, max_iter=100000):
    """Partial sums of Eq. NSum until ||B^{n+1} rho0|| <= tol ||rho0||."""
    rho = rho0.copy()
    term = rho0.copy()
    n0 = np.linalg.norm(rho0)
    for it in range(1, max_iter + 1):
        term = A @ term
        res = np.linalg.norm(term) / n0
        if res <= tol:
            return rho, it, res
        rho = rho + term
    return rho, max_iter, res


def gmres(A, rho0, tol=1e-8, restart=50, max_iter=20000):
    """(I - B) rho = rho0 by scipy's restarted GMRES."""
    n = A.shape[0]
    op = spla.LinearOperator((n, n), matvec=lambda v: v - A @ v, dtype=np.float64)
    rho, info = spla.gmres(op, rho0, rtol=tol, restart=restart, maxiter=max_iter)
    return rho, info
