"""The allocation-free point-source projection (dfm_source_points_noalloc) against
dfm_source_points, through the C ABI: two calls in a row (the second with fewer
points, so stale scratch would show), the size limit, and the error path followed
by a good call on the same scratch."""
import ctypes as C
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_source_points_match_allocating_call():
    from paper_1608_04607_amd import _lib, dfm
    say("[no-alloc] dfm_source_points_noalloc vs dfm_source_points")
    lib = _lib.load()
    v, t = synth.kuhn_box((2, 2, 1), (1.0, 1.0, 0.5), 0.1, 4)
    refl = np.full((t.shape[0], 4), 0.9)
    T = lambda a: torch.tensor(a, device=DEV)  # noqa: E731
    mesh = dfm.Mesh(T(v), T(t), refl=T(refl))
    for order, family, degree in ((1, dfm.LEGENDRE, 6), (0, dfm.ZERNIKE, 4)):
        op = dfm.Operator(mesh, torch.full((t.shape[0],), 0.1, dtype=torch.float64, device=DEV), order, family,
                          degree, 4)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        for ns, seed in ((37, 1), (5, 2)):
            pts = synth.uniform_points_on_box_surface((1.0, 1.0, 0.5), ns, np.random.default_rng(seed))
            xyz = T(pts)
            ref = op.source_points(xyz, flux=0.7)
            out = torch.full((ns, op.ndof), float("nan"), dtype=torch.float64, device=DEV)
            code = lib.dfm_source_points_noalloc(op.handle, C.c_void_p(xyz.data_ptr()), ns, 0.7,
                                                 C.c_void_p(out.data_ptr()), st)
            assert code == 0, lib.dfm_last_error().decode()
            diff = float((out - ref).abs().max() / ref.abs().max())
            say(f"    P{order} family {family} D{degree} ns={ns}: max rel diff {diff:.2e}")
            assert diff <= 1e-14
        # beyond the scratch's size: refused before any device work
        big = torch.zeros((4097, 3), dtype=torch.float64, device=DEV)
        out = torch.empty((1, op.ndof), dtype=torch.float64, device=DEV)
        assert lib.dfm_source_points_noalloc(op.handle, C.c_void_p(big.data_ptr()), 4097, 1.0,
                                             C.c_void_p(out.data_ptr()), st) == -1
        # a point off the boundary is reported, and the next call is right again
        bad = T(np.array([[0.5, 0.5, 0.25]]))
        assert lib.dfm_source_points_noalloc(op.handle, C.c_void_p(bad.data_ptr()), 1, 1.0,
                                             C.c_void_p(out.data_ptr()), st) == -1
        pts = synth.uniform_points_on_box_surface((1.0, 1.0, 0.5), 3, np.random.default_rng(9))
        xyz = T(pts)
        out = torch.empty((3, op.ndof), dtype=torch.float64, device=DEV)
        assert lib.dfm_source_points_noalloc(op.handle, C.c_void_p(xyz.data_ptr()), 3, 1.0,
                                             C.c_void_p(out.data_ptr()), st) == 0
        ref = op.source_points(xyz)
        assert float((out - ref).abs().max() / ref.abs().max()) <= 1e-14
        op.close()
    mesh.close()
