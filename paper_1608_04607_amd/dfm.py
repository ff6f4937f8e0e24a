"""Thin Python binding of the C ABI (include/dfm.h): argument marshalling only.

Device memory and streams come from PyTorch; every computation runs in the HIP
library.  Tensors passed in must be CUDA (HIP) tensors of the documented dtype;
they are made contiguous here and their data pointers handed to the library.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import Basis, SolveInfo, SolveOpts, check

LEGENDRE, ZERNIKE = 0, 1
PAPER_RULE, SEAM_RULE = 0, 1
METHODS = {"neumann": 0, "gmres": 1, "twolevel": 2}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    return t.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Mesh:
    """Face adjacency and geometry of a tetrahedral mesh (dfm_mesh_build)."""

    def __init__(self, verts, tets, refl=None, c=None, rho_f=None, stream=None):
        lib = _lib.load()
        self.verts = _dev(verts, torch.float64)
        self.tets = _dev(tets, torch.int64)
        keep = [self.verts, self.tets]
        args = []
        for a in (refl, c, rho_f):
            a = _dev(a, torch.float64) if a is not None else None
            keep.append(a)
            args.append(_ptr(a))
        self._keep = keep
        h = C.c_void_p()
        check(lib.dfm_mesh_build(_ptr(self.verts), self.verts.shape[0], _ptr(self.tets), self.tets.shape[0],
                                 args[0], args[1], args[2], _stream(stream), C.byref(h)))
        self.handle = h
        self.nt = int(self.tets.shape[0])

    def info(self):
        nt, nb = C.c_int64(), C.c_int64()
        check(_lib.load().dfm_mesh_info(self.handle, C.byref(nt), C.byref(nb)))
        return nt.value, nb.value

    def export(self, stream=None):
        dev = self.verts.device
        nbr = torch.empty((self.nt, 4), dtype=torch.int32, device=dev)
        area = torch.empty((self.nt, 4), dtype=torch.float64, device=dev)
        frame = torch.empty((self.nt, 4, 3, 3), dtype=torch.float64, device=dev)
        vol = torch.empty((self.nt,), dtype=torch.float64, device=dev)
        check(_lib.load().dfm_mesh_export(self.handle, _ptr(nbr), _ptr(area), _ptr(frame), _ptr(vol),
                                          _stream(stream)))
        return nbr, area, frame, vol

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.load().dfm_mesh_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """Assembled transfer operator B (dfm_assemble) and its solves."""

    def __init__(self, mesh: Mesh, mu, pos_order=0, mom_family=LEGENDRE, mom_degree=4, quad_n=8,
                 rule=SEAM_RULE, stream=None, dtype=0):
        lib = _lib.load()
        self.mesh = mesh
        self.mu = _dev(mu, torch.float64)
        self.basis = Basis(pos_order, mom_family, mom_degree, quad_n, rule, int(dtype))
        h = C.c_void_p()
        check(lib.dfm_assemble(mesh.handle, C.byref(self.basis), _ptr(self.mu), _stream(stream), C.byref(h)))
        self.handle = h
        nd, K, nb, nodes, nbytes = (C.c_int64() for _ in range(5))
        check(lib.dfm_op_info(h, C.byref(nd), C.byref(K), C.byref(nb), C.byref(nodes), C.byref(nbytes)))
        self.ndof, self.K, self.nblocks, self.nodes, self.nbytes = nd.value, K.value, nb.value, nodes.value, nbytes.value
        self.device = self.mu.device

    def export(self, stream=None):
        nt = self.mesh.nt
        blocks = torch.empty((nt, 4, 3, self.K, self.K), dtype=torch.float64, device=self.device)
        dest = torch.empty((nt, 4), dtype=torch.int32, device=self.device)
        check(_lib.load().dfm_op_export(self.handle, _ptr(blocks), _ptr(dest), _stream(stream)))
        return blocks, dest

    def export_tets(self, tets, stream=None):
        """Blocks [ns][4][3][K][K] (f64) and dest [ns][4] of the listed tets."""
        tets = _dev(tets, torch.int64)
        if tets.numel() and (int(tets.min()) < 0 or int(tets.max()) >= self.mesh.nt):
            raise ValueError("tet ids must lie in [0, nt)")
        ns = tets.shape[0]
        blocks = torch.empty((ns, 4, 3, self.K, self.K), dtype=torch.float64, device=self.device)
        dest = torch.empty((ns, 4), dtype=torch.int32, device=self.device)
        check(_lib.load().dfm_op_export_tets(self.handle, _ptr(tets), ns, _ptr(blocks), _ptr(dest), _stream(stream)))
        return blocks, dest

    def apply(self, x, transpose=False, stream=None):
        x = _dev(x, torch.float64)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x)
        check(_lib.load().dfm_apply(self.handle, _ptr(x), _ptr(y), nrhs, int(bool(transpose)), _stream(stream)))
        return y

    def apply_f32(self, x, stream=None):
        """y = B32 x for a [nrhs][ndof] FP32 block on the FP32 matrix cores."""
        x = _dev(x, torch.float32)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x)
        check(_lib.load().dfm_apply_f32(self.handle, _ptr(x), _ptr(y), nrhs, _stream(stream)))
        return y

    def apply_f16(self, x, stream=None):
        """y = B16 x for a slot-major FP16 block x [4 nt][nrhs][Kp8] (dfm_apply_f16)."""
        x = _dev(x, torch.float16)
        if x.dim() != 3 or x.shape[0] != 4 * self.mesh.nt or x.shape[2] != (self.K + 7) // 8 * 8:
            raise ValueError("x must be [4 nt][nrhs][Kp8]")
        y = torch.empty_like(x)
        check(_lib.load().dfm_apply_f16(self.handle, _ptr(x), _ptr(y), x.shape[1], _stream(stream)))
        return y

    def product_timing(self, enable=-1):
        """Totals (ms, launches, bytes) of the timed FP16 product launches of method-2
        solves since timing was started, then enable: 1 restart, 0 stop, -1 keep
        (dfm_product_timing)."""
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        check(_lib.load().dfm_product_timing(self.handle, int(enable), C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def solve(self, rho0, method="gmres", rtol=1e-8, restart=50, max_iter=20000, precision=0, stream=None,
              raise_nonconv=True, rho=None):
        """Solve (I - B) rho = rho0 with method "neumann", "gmres" or "twolevel" (the
        batched two-level iteration, FP16 products inside FP64 refinement: precision
        2); `rho` given: start from it (batched methods only) and write the result
        into it."""
        m = METHODS[method]
        if m == 2:
            precision = 2
        rho0 = _dev(rho0, torch.float64)
        nrhs = 1 if rho0.dim() == 1 else rho0.shape[0]
        warm = rho is not None
        if warm:
            if rho.shape != rho0.shape or rho.dtype != torch.float64 or not rho.is_cuda or not rho.is_contiguous():
                raise TypeError("rho must be a contiguous CUDA float64 tensor shaped like rho0")
        else:
            rho = torch.empty_like(rho0)
        opts = SolveOpts(m, restart, max_iter, rtol, int(precision), int(warm))
        info = (SolveInfo * nrhs)()
        code = _lib.load().dfm_solve(self.handle, _ptr(rho0), _ptr(rho), nrhs, C.byref(opts), info, _stream(stream))
        if code != 0 and (raise_nonconv or code != -5):
            check(code)
        return rho, [(i.iters, i.restarts, i.relres) for i in info]

    def solve_groups(self, rho0, tet_offsets, rtol=1e-8, max_iter=20000, stream=None, raise_nonconv=True, rho=None,
                     method="neumann"):
        """Batched solve of independent instances packed into this operator
        (dfm_solve_groups): instance g owns tets [tet_offsets[g], tet_offsets[g+1]).
        method "neumann" (FP32 Neumann, precision 1) or "twolevel" (precision 2).
        Returns rho and info [ngroups][nrhs] of (iters, restarts, relres)."""
        rho0 = _dev(rho0, torch.float64)
        nrhs = 1 if rho0.dim() == 1 else rho0.shape[0]
        warm = rho is not None
        if warm:
            if rho.shape != rho0.shape or rho.dtype != torch.float64 or not rho.is_cuda or not rho.is_contiguous():
                raise TypeError("rho must be a contiguous CUDA float64 tensor shaped like rho0")
        else:
            rho = torch.empty_like(rho0)
        G = len(tet_offsets) - 1
        offs = (C.c_int64 * (G + 1))(*[int(v) for v in tet_offsets])
        m = METHODS[method]
        if m == 1:
            raise ValueError("instance groups are solved with method 'neumann' or 'twolevel'")
        opts = SolveOpts(m, 1, max_iter, rtol, 2 if m == 2 else 1, int(warm))
        info = (SolveInfo * (G * nrhs))()
        code = _lib.load().dfm_solve_groups(self.handle, _ptr(rho0), _ptr(rho), nrhs, C.byref(opts), offs, G, info,
                                            _stream(stream))
        if code != 0 and (raise_nonconv or code != -5):
            check(code)
        out = [[(info[g * nrhs + r].iters, info[g * nrhs + r].restarts, info[g * nrhs + r].relres)
                for r in range(nrhs)] for g in range(G)]
        return rho, out

    def residual(self, rho0, rho, stream=None):
        """rho0 - (I - B) rho for one or several right-hand sides (dfm_residual)."""
        rho0, rho = _dev(rho0, torch.float64), _dev(rho, torch.float64)
        if rho0.shape != rho.shape:
            raise ValueError("rho0 and rho must have the same shape")
        nrhs = 1 if rho0.dim() == 1 else rho0.shape[0]
        res = torch.empty_like(rho0)
        check(_lib.load().dfm_residual(self.handle, _ptr(rho0), _ptr(rho), _ptr(res), nrhs, _stream(stream)))
        return res

    def source_points(self, xyz, flux=1.0, stream=None):
        xyz = _dev(xyz, torch.float64)
        ns = xyz.shape[0]
        rho0 = torch.empty((ns, self.ndof), dtype=torch.float64, device=self.device)
        check(_lib.load().dfm_source_points(self.handle, _ptr(xyz), ns, flux, _ptr(rho0), _stream(stream)))
        return rho0

    def source_points_sum(self, xyz, which, nrhs, flux=1.0, stream=None):
        """Point sources summed into nrhs right-hand sides: rho0[which[i]] += point i."""
        xyz = _dev(xyz, torch.float64)
        which = _dev(which, torch.int32)
        rho0 = torch.empty((nrhs, self.ndof), dtype=torch.float64, device=self.device)
        check(_lib.load().dfm_source_points_sum(self.handle, _ptr(xyz), xyz.shape[0], _ptr(which), int(nrhs), flux,
                                                _ptr(rho0), _stream(stream)))
        return rho0

    def source_plane(self, axis, value, profile=0, params=None, flux=1.0, stream=None):
        rho0 = torch.empty((self.ndof,), dtype=torch.float64, device=self.device)
        par = (C.c_double * 4)(*(params if params is not None else (0.0, 0.0, 0.0, 1.0)))
        check(_lib.load().dfm_source_plane(self.handle, axis, float(value), profile, par, flux, _ptr(rho0),
                                           _stream(stream)))
        return rho0

    def receiver_functional(self, box, stream=None):
        g = torch.empty((self.ndof,), dtype=torch.float64, device=self.device)
        bx = (C.c_double * 6)(*box)
        check(_lib.load().dfm_receiver_functional(self.handle, _ptr(self.mu), bx, _ptr(g), _stream(stream)))
        return g

    def receiver_energy(self, rho, box, stream=None):
        """J = g . rho (one value per row of rho) for the receiver box (dfm_receiver_energy)."""
        rho = _dev(rho, torch.float64)
        nrhs = 1 if rho.dim() == 1 else rho.shape[0]
        J = torch.empty((nrhs,), dtype=torch.float64, device=self.device)
        bx = (C.c_double * 6)(*box)
        check(_lib.load().dfm_receiver_energy(self.handle, _ptr(self.mu), bx, _ptr(rho), nrhs, _ptr(J),
                                              _stream(stream)))
        return J

    def adjoint(self, rho, box, src=None, method="gmres", rtol=1e-10, restart=50, max_iter=20000, precision=0,
                stream=None):
        """(lambda, dJ/dmu, dJ/dw, info) for J = receiver energy in `box`; precision 1:
        FP32 GMRES corrections inside FP64 refinement for the transposed solve."""
        rho = _dev(rho, torch.float64)
        nsrc = 0 if src is None else src.shape[0]
        src = _dev(src, torch.float64) if src is not None else None
        lam = torch.empty((self.ndof,), dtype=torch.float64, device=self.device)
        dmu = torch.empty((self.mesh.nt,), dtype=torch.float64, device=self.device)
        dw = torch.empty((max(nsrc, 1),), dtype=torch.float64, device=self.device)
        bx = (C.c_double * 6)(*box)
        opts = SolveOpts(1 if method == "gmres" else 0, restart, max_iter, rtol, int(precision), 0)
        info = SolveInfo()
        check(_lib.load().dfm_adjoint(self.handle, _ptr(self.mu), bx, _ptr(rho), _ptr(src), nsrc, C.byref(opts),
                                      _ptr(lam), _ptr(dmu), _ptr(dw), C.byref(info), _stream(stream)))
        return lam, dmu, dw[:nsrc], (info.iters, info.restarts, info.relres)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.load().dfm_op_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def weighted_sum(x, w, stream=None):
    """y = sum_s w[s] x[s] for x [nvec][n] and w [nvec] (dfm_weighted_sum)."""
    x = _dev(x, torch.float64)
    w = _dev(w, torch.float64)
    nvec = 1 if x.dim() == 1 else x.shape[0]
    if w.numel() != nvec:
        raise ValueError("w needs one weight per row of x")
    y = torch.empty((x.shape[-1],), dtype=torch.float64, device=x.device)
    check(_lib.load().dfm_weighted_sum(_ptr(x), x.shape[-1], nvec, _ptr(w), _ptr(y), _stream(stream)))
    return y


class ReceiverEnergy(torch.autograd.Function):
    """J(mu, w) = receiver energy in `box` of the stationary density for the source
    rho0 = sum_s w_s src_s, differentiable in the damping mu [nt] and the source
    weights w [nsrc].  Forward: dfm_assemble (for this mu), dfm_weighted_sum,
    dfm_solve, dfm_receiver_energy; backward: dfm_adjoint (transposed solve and
    the dB/dmu contraction), scaled by the incoming gradient with dfm_weighted_sum."""

    @staticmethod
    def forward(ctx, mu, w, mesh, src, box, basis, rtol=1e-12, restart=50):
        pos_order, family, degree, quad_n, rule = basis
        op = Operator(mesh, mu.detach(), pos_order, family, degree, quad_n, rule=rule)
        rho0 = weighted_sum(src, w.detach().to(torch.float64))
        rho, _ = op.solve(rho0, method="gmres", rtol=rtol, restart=restart)
        J = op.receiver_energy(rho, box)
        ctx.save_for_backward(rho)
        ctx.op, ctx.src, ctx.box, ctx.rtol, ctx.restart = op, src, box, rtol, restart
        return J.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (rho,) = ctx.saved_tensors
        op = ctx.op
        _, dmu, dw, _ = op.adjoint(rho, ctx.box, src=ctx.src, rtol=ctx.rtol, restart=ctx.restart)
        op.close()
        scale = grad_out.detach().to(torch.float64).reshape(1)
        return weighted_sum(dmu, scale), weighted_sum(dw, scale), None, None, None, None, None, None


def receiver_energy(mesh, mu, w, src, box, basis, rtol=1e-12, restart=50):
    """Differentiable receiver energy (see ReceiverEnergy); basis = (pos_order,
    mom_family, mom_degree, quad_n, rule)."""
    return ReceiverEnergy.apply(mu, w, mesh, src, tuple(box), tuple(basis), rtol, restart)

