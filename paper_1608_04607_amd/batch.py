"""Uneven batches of independent instances: meshes of different sizes, with their own
damping, wall coefficients, momentum degree and point sources, solved together.

Instances that share a discretisation (position order, momentum family and degree,
Gauss points) are concatenated into one mesh.  Its components are disjoint, so B is
block diagonal and one dfm_assemble launch assembles every instance of the group;
right-hand side s of the group carries the s-th source of every instance
(dfm_source_points_sum), and one batched solve (dfm_solve_groups: by default the
two-level iteration with FP16 products inside FP64 refinement, or Neumann with
FP32 corrections) solves all of them, each instance and source stopping on its
own residual and each instance leaving the products once all its sources have
converged.
This module only arranges arrays and calls the library; every step of the method
runs in its kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import dfm


@dataclass
class Group:
    key: tuple                       # (pos_order, mom_family, mom_degree, quad_n)
    members: list                    # instance indices
    tet_offsets: list                # first tet of every member in the group mesh (+ total)
    nsrc: int
    K: int = 0                       # unknowns per slot (kept after the operator is released)
    mesh: dfm.Mesh = None
    op: dfm.Operator = None
    rho0: torch.Tensor = None
    rho: torch.Tensor = None
    products: int = 0                # batched product launches
    member_products: list = field(default_factory=list)   # products that included each member
    relres: list = field(default_factory=list)   # [member][rhs] on the member's own residual
    t_assembled: float = 0.0         # host time when the group's operator was ready
    events: list = field(default_factory=list)   # timing events of assemble()


class UnevenBatch:
    """problems: objects with verts, tets, mu, refl, pos_order, mom_degree, quad_n and
    source = {"kind": "points", "xyz": ...} (e.g. synth.problem_c5())."""

    def __init__(self, problems, mom_family=dfm.LEGENDRE, rule=dfm.SEAM_RULE, dtype=1, device="cuda:0",
                 method="twolevel"):
        self.problems = list(problems)
        self.method = method
        self.family, self.rule, self.dtype, self.device = mom_family, rule, dtype, torch.device(device)
        ext = [p.verts.max(axis=0) - p.verts.min(axis=0) for p in self.problems]
        self._gap = 1.5 * max(float(e[0]) for e in ext) + 0.5    # x spacing of the instance grid
        self._row = 1.5 * max(float(e[1]) for e in ext) + 0.5    # y spacing of its rows
        groups = {}
        for i, p in enumerate(self.problems):
            groups.setdefault((p.pos_order, mom_family, p.mom_degree, p.quad_n), []).append(i)
        self.groups = []
        for key in sorted(groups):
            mem = groups[key]
            offs = [0]
            for i in mem:
                offs.append(offs[-1] + self.problems[i].nt)
            nsrc = max(len(self.problems[i].source["xyz"]) for i in mem)
            self.groups.append(Group(key, mem, offs, nsrc))

    def _concat(self, g):
        T = lambda a, dt: torch.as_tensor(a, dtype=dt).to(self.device)  # noqa: E731
        verts, tets, mu, refl, xyz, which = [], [], [], [], [], []
        voff = 0
        for m, i in enumerate(g.members):
            p = self.problems[i]
            # instances are moved apart (the transport is translation invariant) so
            # that a source point is found on its own instance's boundary
            lo, hi = p.verts.min(axis=0), p.verts.max(axis=0)
            shift = torch.tensor([self._gap * (m % 16) - lo[0], self._row * (m // 16) - lo[1], -lo[2]],
                                 dtype=torch.float64, device=self.device)
            verts.append(T(p.verts, torch.float64) + shift)
            tets.append(T(p.tets, torch.int64) + voff)
            mu.append(T(p.mu, torch.float64))
            refl.append(T(p.refl, torch.float64))
            pts = T(p.source["xyz"], torch.float64) + shift
            xyz.append(pts)
            which.append(torch.arange(pts.shape[0], dtype=torch.int32, device=self.device))
            voff += p.verts.shape[0]
        cat = torch.cat
        return cat(verts), cat(tets), cat(mu), cat(refl), cat(xyz), cat(which)

    def assemble(self, g, stream=None):
        """Mesh, operator and right-hand sides of group g; g.events brackets the mesh
        build + assembly and the source projection on `stream` (for timing)."""
        verts, tets, mu, refl, xyz, which = self._concat(g)
        pos_order, family, degree, quad_n = g.key
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        g.events = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        g.events[0].record(st)
        g.mesh = dfm.Mesh(verts, tets, refl=refl, stream=stream)
        g.op = dfm.Operator(g.mesh, mu, pos_order, family, degree, quad_n, rule=self.rule, stream=stream,
                            dtype=self.dtype)
        g.K = g.op.K
        g.events[1].record(st)
        g.rho0 = g.op.source_points_sum(xyz, which, g.nsrc, stream=stream)
        g.events[2].record(st)

    def solve(self, g, rtol=1e-8, segment=2500, max_products=100000, progress=None, stream=None, method=None):
        """Solve the group to relative residual rtol on every instance and source
        (dfm_solve_groups), in warm-started segments of at most `segment` batched
        products; instances stop being multiplied once all their sources converged."""
        while True:
            g.rho, info = g.op.solve_groups(g.rho0, g.tet_offsets, rtol=rtol, max_iter=segment, rho=g.rho,
                                            raise_nonconv=False, stream=stream, method=method or self.method)
            g.products += max(x[0] for row in info for x in row)
            if not g.member_products:
                g.member_products = [0] * len(g.members)
            for m, row in enumerate(info):
                g.member_products[m] += row[0][0]
            g.relres = [[x[2] for x in row] for row in info]
            worst = max(max(r) for r in g.relres)
            if progress:
                progress(g, worst)
            if worst <= rtol or g.products >= max_products:
                return

    def solve_all(self, rtol=1e-8, segment=2500, max_products=100000, overlap=False, progress=None, on_group=None):
        """Assemble and solve every group, releasing each group's operator after its
        solve.  With overlap, group g + 1 is assembled on a second stream (from a second
        host thread, since dfm_assemble waits for its kernels) while group g is solved.
        Both phases fill every compute unit, so on the 256-box batch this saves only
        about 1 % of the wall time (the solve slows by what the assembly takes).  on_group(g, t) is called
        after each group's solve (and after the next group's assembly has finished)
        with the solve's host time in ms, before the group is released."""
        import threading
        import time

        main = torch.cuda.current_stream(self.device)
        side = torch.cuda.Stream(self.device) if overlap else main
        err = []

        def build(g):
            try:
                with torch.cuda.stream(side):
                    self.assemble(g, stream=side)
                side.synchronize()
                g.t_assembled = time.perf_counter()
            except Exception as e:  # reported on the main thread
                err.append(e)

        groups = list(self.groups)
        if not groups:
            return
        build(groups[0])
        for k, g in enumerate(groups):
            if err:
                raise err[0]
            worker = None
            if overlap and k + 1 < len(groups):
                worker = threading.Thread(target=build, args=(groups[k + 1],))
                worker.start()
            try:
                # group g's assembly finished before build() returned (side.synchronize()),
                # so the solve on the main stream needs no event wait on the side stream
                t0 = time.perf_counter()
                self.solve(g, rtol=rtol, segment=segment, max_products=max_products, progress=progress,
                           stream=main)
                main.synchronize()
                t_solve = (time.perf_counter() - t0) * 1e3
            finally:
                if worker is not None:
                    worker.join()  # also when the solve raised; on_group then has the GPU to itself
            if on_group:
                on_group(g, t_solve)
            self.release(g)
            g.rho0 = None
            torch.cuda.empty_cache()
            if worker is None and k + 1 < len(groups):
                build(groups[k + 1])
        if err:
            raise err[0]

    def solution(self, i):
        """rho of instance i: [nsrc][4 nt K] (the group's rhs s is the instance's source s)."""
        for g in self.groups:
            if i in g.members:
                m = g.members.index(i)
                K = g.K
                return g.rho[:, 4 * K * g.tet_offsets[m]:4 * K * g.tet_offsets[m + 1]]
        raise KeyError(i)

    def release(self, g):
        if g.op is not None:
            g.op.close()
        if g.mesh is not None:
            g.mesh.close()
        g.op = g.mesh = None
