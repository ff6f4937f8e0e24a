"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, undone after the case)
and checks that a pin which the unmodified oracle passes now fails by a wide
margin:

* Monte Carlo ray tracing of whole blocks (independent tracer, tests/refgeom.py)
  against a dropped or sign-flipped attenuation exp(-mu L) (Sec. 3.3, the
  chord integral), a forgotten wall reflection (Sec. 2, the specular map), and
  an azimuth measured from the wrong frame axis (Sec. 3.3, the local face frame),
  and direction weights of the solid angle instead of the flux measure (Sec. 3.4);
* the stationary energy balance of the cube (Sec. 2: with mu = 0 and R = 1 on
  every wall but the absorbing one, all injected density leaves through that
  face) against the wall coefficient applied on interior faces and a dropped
  Gram solve (Eq. Bapprox);
* flux conservation of a lossless tet (Sec. 2) against the dropped Gram solve
  and the solid-angle weights;
* central differences of the receiver energy against the adjoint gradient with
  the sign of dB/dmu flipped, the wall coefficient left out of dB/dmu, or the
  receiver functional's own dependence on mu dropped.
"""
import math

import numpy as np
import pytest

import synth
import oracle.assemble as oas
from oracle import adjoint as oj
from oracle import assemble as oa
from oracle import basis as ob
from oracle import geometry as og
from oracle import mesh as om
from oracle import quadrature as oq
from oracle import solve as osv
from oracle import sources as osrc
from tests import refgeom as rg

MC_Z = 5.5            # the Monte Carlo pin's bound (standard errors)
BALANCE_REL = 1e-4    # the energy-balance pin's bound
CONSERVATION = 1e-9   # the conservation pin's bound (Zernike, paper rule)
FD_REL = 1e-6         # the central-difference pin's bound on dJ/dmu


@pytest.fixture(scope="module")
def jmesh():
    p = synth.problem_c2(n_cells=2)
    return om.build_mesh(p.verts, p.tets, p.refl)


def mc_z(jm, order, mu, case, nrays=300_000, seed=7):
    """Largest |T - MC| in standard errors over the block (D = 3, seam rule)."""
    j, li, lo = case
    bs = oa.Basis(order, ob.LEGENDRE, 3, 24, oq.SEAM_RULE)
    T, slot, _ = oa.block_T(jm, bs, mu, j, li, lo)
    transmitted = jm.nbr[j, lo] >= 0
    dest = rg.face_frame(jm.verts, jm.tets[slot // 4], slot % 4)
    X, se = rg.mc_block(jm.verts, jm.tets[j], li, lo, mu, 3, order, nrays, np.random.default_rng(seed),
                        dest_frame=dest, reflect=not transmitted)
    return float((np.abs(T - X) / np.maximum(se, 1e-6 * np.abs(T).max())).max())


def interior_case(jm):
    return next((j, li, lo) for j in range(jm.nt) for lo in range(4) for li in range(4)
                if li != lo and jm.nbr[j, lo] >= 0)


def wall_case(jm):
    return next((j, li, lo) for j in range(jm.nt) for lo in range(4) for li in range(4)
                if li != lo and jm.nbr[j, lo] < 0)


def balance_error():
    """Relative mismatch of injected and absorbed density on the one-cell cube."""
    c = synth.problem_c1()
    m = om.build_mesh(c.verts, c.tets, c.refl)
    bs = oa.Basis(c.pos_order, ob.LEGENDRE, c.mom_degree, c.quad_n, oq.SEAM_RULE)
    B, dest = oa.assemble(m, bs, c.mu)
    rho0 = osrc.project(m, bs, c.source)[0]
    rho = osv.solve_direct(osv.to_sparse(B, dest), rho0)
    full = synth.Problem(**{**c.__dict__, "refl": np.ones_like(c.refl)})
    Bf, _ = oa.assemble(om.build_mesh(full.verts, full.tets, full.refl), bs, full.mu)
    G = ob.gram(bs.mom_degree, bs.mom_family)
    mv = np.zeros((4 * m.nt, bs.P, bs.M))
    mv[:, 0, :] = np.sqrt(m.area.reshape(-1))[:, None] * G[:, 0][None, :]
    mv = mv.reshape(4 * m.nt, -1)
    y = osv.apply(Bf, dest, rho).reshape(4 * m.nt, bs.K)
    absorbed = sum(mv[s] @ y[s] for s in range(4 * m.nt) if m.nbr[s // 4, s % 4] < 0 and m.refl[s // 4, s % 4] == 0)
    injected = mv.ravel() @ rho0
    return abs(absorbed - injected) / abs(injected)


def conservation_error(jm):
    D = 6
    bs = oa.Basis(1, ob.ZERNIKE, D, 32, oq.PAPER_RULE)
    G = ob.gram(D, ob.ZERNIKE)
    err = 0.0
    for (j, li) in [(5, 0), (22, 3)]:
        tot = np.zeros(bs.K)
        for lo in range(4):
            if lo != li:
                T, _, _ = oa.block_T(jm, bs, 0.0, j, li, lo)
                tot += math.sqrt(jm.area[j, lo]) * T[0]
        ref = np.zeros(bs.K)
        ref[:bs.M] = math.sqrt(jm.area[j, li]) * G[:, 0]
        err = max(err, np.abs(tot - ref).max() / np.abs(ref).max())
    return err


def fd_error():
    """Largest relative gap between the adjoint dJ/dmu_e and central differences
    of J = g . rho on a 12-tet box with walls R = 0.8 (three elements e)."""
    v, t = synth.kuhn_box((2, 1, 1), (1.0, 1.0, 1.0), 0.15, 3)
    refl = np.full((t.shape[0], 4), 0.8)
    mu = np.random.default_rng(1).uniform(0.1, 0.6, t.shape[0])
    bs = oa.Basis(1, 0, 2, 4, oq.SEAM_RULE)
    box = (0.5, 1.0, 0.0, 1.0, 0.0, 0.7)
    src = {"kind": "points", "xyz": synth.uniform_points_on_box_surface((1, 1, 1), 3, np.random.default_rng(2))}
    m = om.build_mesh(v, t, refl)
    rho0 = osrc.project(m, bs, src).sum(0)

    def J(mu_):
        B, dest = oa.assemble(m, bs, mu_)
        return oj.receiver_functional(m, bs, mu_, box) @ osv.solve_direct(osv.to_sparse(B, dest), rho0)

    B, dest = oa.assemble(m, bs, mu)
    A = osv.to_sparse(B, dest)
    rho = osv.solve_direct(A, rho0)
    lam = osv.solve_direct(A.T.tocsr(), oj.receiver_functional(m, bs, mu, box))
    dmu = oj.gradient_mu(m, bs, mu, lam, rho, box)
    h, err = 1e-6, 0.0
    for e in (0, 7, 10):
        mp, mm = mu.copy(), mu.copy()
        mp[e] += h
        mm[e] -= h
        fd = (J(mp) - J(mm)) / (2 * h)
        err = max(err, abs(dmu[e] - fd) / max(abs(fd), 1e-9 * np.abs(dmu).max()))
    return err


_g, _m, _dest, _gram, _ang = og.g_exp, og.moment_I, oas.destination, ob.gram, ob.direction_angles
_nodes = oq.block_nodes
_dB, _jdest, _recv = oj.dB_dmu_block, oj.destination, oj.receiver_functional


def _plant(monkeypatch, name):
    if name == "no_attenuation":
        monkeypatch.setattr(og, "g_exp", lambda a: _g(0.0 * a))
        monkeypatch.setattr(og, "moment_I", lambda i, m, a: _m(i, m, 0.0 * a))
    elif name == "attenuation_sign":
        monkeypatch.setattr(og, "g_exp", lambda a: _g(-a))
        monkeypatch.setattr(og, "moment_I", lambda i, m, a: _m(i, m, -a))
    elif name == "no_reflection":
        monkeypatch.setattr(oas, "destination", lambda mesh, j, lo: (lambda r: (r[0], True, r[2], r[3]))(_dest(mesh, j, lo)))
    elif name == "wall_weight_on_interior":
        monkeypatch.setattr(oas, "destination",
                            lambda mesh, j, lo: (lambda r: (r[0], r[1], 0.9 if r[1] else r[2], r[3]))(_dest(mesh, j, lo)))
    elif name == "no_gram_solve":
        monkeypatch.setattr(ob, "gram", lambda D, f: np.eye(_gram(D, f).shape[0]))
    elif name == "azimuth_from_y_axis":
        monkeypatch.setattr(ob, "direction_angles",
                            lambda d, fr: (lambda ct, ph: (ct, (ph - 0.5 * np.pi) % (2 * np.pi)))(*_ang(d, fr)))
    elif name == "solid_angle_weights":
        # d Omega instead of the flux measure cos(theta) d Omega (Sec. 3.4)
        monkeypatch.setattr(oq, "block_nodes", lambda mesh, j, li, lo, n, rule=oq.PAPER_RULE: (
            lambda d, w: (d, w / np.abs(d @ mesh.frame[j, li, 2])))(*_nodes(mesh, j, li, lo, n, rule)))
    elif name == "dB_dmu_sign":
        monkeypatch.setattr(oj, "dB_dmu_block", lambda *a: (lambda r: (-r[0], r[1]))(_dB(*a)))
    elif name == "wall_weight_missing_in_dB_dmu":
        monkeypatch.setattr(oj, "destination", lambda mesh, j, lo: (lambda r: (r[0], r[1], 1.0, r[3]))(_jdest(mesh, j, lo)))
    elif name == "receiver_mu_dependence_dropped":
        monkeypatch.setattr(oj, "receiver_functional",
                            lambda mesh, bs, mu, box, derivative=False:
                            0.0 * _recv(mesh, bs, mu, box, True) if derivative else _recv(mesh, bs, mu, box))
    else:
        assert name == "none"


def test_unmodified_oracle_passes_the_detectors(jmesh):
    assert mc_z(jmesh, 0, 0.8, interior_case(jmesh)) < MC_Z
    assert mc_z(jmesh, 1, 0.8, wall_case(jmesh)) < MC_Z
    assert balance_error() < BALANCE_REL
    assert conservation_error(jmesh) < CONSERVATION
    assert fd_error() < FD_REL


@pytest.mark.parametrize("name,detector", [
    ("no_attenuation", "mc_interior"),
    ("attenuation_sign", "mc_interior"),
    ("no_reflection", "mc_wall"),
    ("azimuth_from_y_axis", "mc_interior"),
    ("wall_weight_on_interior", "balance"),
    ("no_gram_solve", "balance"),
    ("no_gram_solve", "conservation"),
    ("solid_angle_weights", "conservation"),
    ("solid_angle_weights", "mc_interior"),
    ("dB_dmu_sign", "fd"),
    ("wall_weight_missing_in_dB_dmu", "fd"),
    ("receiver_mu_dependence_dropped", "fd"),
])
def test_planted_mistake_is_caught(jmesh, monkeypatch, name, detector):
    _plant(monkeypatch, name)
    if detector == "mc_interior":
        assert mc_z(jmesh, 0, 0.8, interior_case(jmesh)) > 4 * MC_Z
    elif detector == "mc_wall":
        assert mc_z(jmesh, 1, 0.8, wall_case(jmesh)) > 4 * MC_Z
    elif detector == "balance":
        assert balance_error() > 10 * BALANCE_REL
    elif detector == "fd":
        assert fd_error() > 1e3 * FD_REL
    else:
        assert conservation_error(jmesh) > 1e6 * CONSERVATION
