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
