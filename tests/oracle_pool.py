"""Oracle work run in worker processes (spawned fresh, so they never touch the GPU
of the test process): whole-instance assembly, source projection and direct solve."""
import os

os.environ.setdefault("OMP_NUM_THREADS", "1")

import numpy as np  # noqa: E402

from oracle import assemble as oa  # noqa: E402
from oracle import mesh as om  # noqa: E402
from oracle import solve as osv  # noqa: E402
from oracle import sources as osrc  # noqa: E402


def instance_solution(args):
    """(B [nt][4][3][K][K], dest, rho [nsrc][ndof]) of one problem: the oracle's
    blocks, its point sources and the sparse-LU solution of (I - B) rho = rho0."""
    verts, tets, refl, mu, pos_order, family, degree, quad_n, rule, xyz = args
    m = om.build_mesh(verts, tets, refl)
    bs = oa.Basis(pos_order, family, degree, quad_n, rule)
    B, dest = oa.assemble(m, bs, mu)
    rho0 = osrc.project(m, bs, {"kind": "points", "xyz": xyz})
    A = osv.to_sparse(B, dest)
    rho = np.stack([osv.solve_direct(A, r) for r in rho0])
    return B, dest, rho


def pool_map(fn, items, workers=None):
    import multiprocessing as mp
    workers = workers or min(len(items), max(1, min(16, len(os.sched_getaffinity(0)))))
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(fn, items)


def tet_blocks(args):
    """The oracle's blocks and destination slots of the listed tets of one mesh."""
    verts, tets, refl, mu, pos_order, family, degree, quad_n, rule, which = args
    m = om.build_mesh(verts, tets, refl)
    bs = oa.Basis(pos_order, family, degree, quad_n, rule)
    return oa.assemble(m, bs, mu, tets=which)


def tet_dB_terms(args):
    """lambda^T (dB/dmu_j) rho summed over the 12 blocks of each listed tet j (the
    oracle's block derivative, as in its gradient_mu)."""
    from oracle import adjoint as oj
    from oracle.assemble import in_faces
    verts, tets, refl, mu, pos_order, family, degree, quad_n, rule, which, lam, rho = args
    m = om.build_mesh(verts, tets, refl)
    bs = oa.Basis(pos_order, family, degree, quad_n, rule)
    K = bs.K
    lam = lam.reshape(4 * m.nt, K)
    rr = rho.reshape(4 * m.nt, K)
    out = []
    for j in which:
        acc = 0.0
        for l_out in range(4):
            for l_in in in_faces(l_out):
                dB, slot = oj.dB_dmu_block(m, bs, mu[j], j, l_in, l_out)
                acc += lam[slot] @ dB @ rr[4 * j + l_in]
        out.append(acc)
    return out
