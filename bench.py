"""Benchmark of the discrete flow mapping hot path on one MI355X.

Default workload: the batched 49152-tetrahedron box (2 x 1 x 1, 32x16x16 Kuhn
cells, jitter 0.1h, piecewise-constant position basis x Legendre momentum basis
of degree 12, 16-point Gauss rule per cell, lognormal damping, walls R = 0.9,
128 isotropic boundary point sources).  One step is the whole path:
    mesh build -> FP64 assembly of B -> projection of the 128 sources -> the
    two-level solve of all 128 right-hand sides to relative residual 1e-8
(coloured Gauss-Seidel sweeps with a coarse correction, FP16 products on the
matrix cores, FP64 refinement residuals of the stored operator).  Inputs are
resident in HBM before the timed region starts.

After the timed steps, on the last step's operator: true FP64 residuals of three
of its solutions, the batched FP64 product (dfm_residual) for an estimate of plain
FP64 solving all 128 at once, and one plain FP64 Neumann solve of source 0, the
per-right-hand-side reference.

Prints ONE JSON line.  `value` is B-assembly face-pair blocks per second (12 per
tet) over the timed steps; the solve's ms per right-hand side and its ratio to
plain FP64 are reported beside it.  `roofline` is the kernel with the most time
per step: the FP16 product of the sweeps (timed per launch with HIP events on the
solve's stream, dfm_product_timing) or the assembly; `cpu_baseline` is the CPU
oracle timed on bounded samples of the same workload on this host, before the GPU
is touched.  Other workloads: --workload box8 (3072 tets, one right-hand side),
box32-adjoint, uneven.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "B-assembly face-pair blocks/s; (I-B)rho solve ms/RHS at 1e-8 residual vs plain FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rule", choices=["seam", "paper"], default="seam")
    ap.add_argument("--workload", choices=["box8", "box32-batched", "box32-adjoint", "uneven"],
                    default="box32-batched",
                    help="box32-batched: 49152 tets, 128 sources (default); box8: the 3072-tet single-rhs case; "
                         "box32-adjoint: receiver-energy gradients on the same box (64 sources); "
                         "uneven: 256 independent boxes of 384-20412 tets, degrees 4-10, 4 sources each")
    ap.add_argument("--instances", type=int, default=256, help="uneven: number of boxes")
    ap.add_argument("--overlap", action="store_true",
                    help="uneven: assemble the next group on a second stream beside the current solve "
                         "(per-group assembly times then include the contention)")
    ap.add_argument("--fp64-sample", type=int, default=2,
                    help="uneven: boxes per degree solved one by one in plain FP64 for the comparison")
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--cpu-tets", type=int, default=24, help="tets in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="box32-batched: skip the plain FP64 single-rhs reference solve after the steps")
    ap.add_argument("--copy-calib", action="store_true", help="only run a plain device copy of known size")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only one assembly and five products with B (for hardware counters)")
    return ap.parse_args()


# --------------------------------------------------------------------------- CPU oracle baseline

_ORACLE = {}


def _oracle_init(verts, tets, refl, rule, pos_order=1, degree=8, quad_n=12):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import assemble as oa
    from oracle import mesh as om
    _ORACLE["mesh"] = om.build_mesh(verts, tets, refl)
    _ORACLE["bs"] = oa.Basis(pos_order, 0, degree, quad_n, rule)


def _oracle_tet(args):
    j, mu = args
    from oracle import assemble as oa
    oa.assemble(_ORACLE["mesh"], _ORACLE["bs"], mu, tets=[j])
    return 12


def _oracle_blocks(prob, rule, ntets, seed=6):
    """(blocks, seconds, cores) of the unmodified oracle assembling `ntets` tets of
    `prob` drawn with `seed`, one worker process per core."""
    import multiprocessing as mp

    import numpy as np
    cores = min(16, len(os.sched_getaffinity(0)))
    sample = np.random.default_rng(seed).choice(prob.nt, min(ntets, prob.nt), replace=False)
    ctx = mp.get_context("fork")
    init = (prob.verts, prob.tets, prob.refl, rule, prob.pos_order, prob.mom_degree, prob.quad_n)
    with ctx.Pool(cores, initializer=_oracle_init, initargs=init) as pool:
        pool.map(_oracle_tet, [(int(sample[0]), prob.mu)] * cores)      # warm every worker
        t0 = time.perf_counter()
        blocks = sum(pool.map(_oracle_tet, [(int(j), prob.mu) for j in sample], chunksize=1))
        dt = time.perf_counter() - t0
    return blocks, dt, cores


def cpu_baseline(prob, rule, ntets, label="3072-tet box"):
    """Blocks/s of the unmodified oracle on `ntets` sampled tets, one process per core
    (at most 16, the CPU share of one GPU; `host_cpus` is what the host offers)."""
    blocks, dt, cores = _oracle_blocks(prob, rule, ntets)
    return {"value": blocks / dt, "unit": "blocks/s", "cores": cores, "host_cpus": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"{ntets} tets ({blocks} blocks) drawn with seed 6 from the same {label}, "
                      f"FP64 NumPy oracle, {cores} worker processes, {dt:.1f} s"}


def oracle_product_ms(sub, K, full_nt, seed=7, min_s=1.0):
    """The oracle's y = B x (its SciPy CSR operator, FP64, one thread) on the sub-box
    `sub` (the workload's recipe on fewer cells), with random blocks of size K (the
    time does not depend on the values), scaled to `full_nt` tets by the operator's
    size.  Returns (ms per product at full size, ms on the sub-box, sub-box tets)."""
    import numpy as np
    from oracle import mesh as om
    from oracle import solve as osv
    M = om.build_mesh(sub.verts, sub.tets, sub.refl)
    dest = np.array([[om.destination(M, j, l)[0] for l in range(4)] for j in range(sub.nt)], dtype=np.int64)
    rng = np.random.default_rng(seed)
    B = rng.uniform(0.0, 1.0 / (3 * K), size=(sub.nt, 4, 3, K, K))
    A = osv.to_sparse(B, dest)
    del B
    x = rng.standard_normal(A.shape[0])
    A @ x
    n, t0 = 0, time.perf_counter()
    while True:
        A @ x
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_s and n >= 3:
            break
    ms_sub = dt / n * 1e3
    return ms_sub * full_nt / sub.nt, ms_sub, sub.nt


# --------------------------------------------------------------------------- HBM byte counters

COUNTERS = os.path.join(ROOT, "profiles", "counters_box8x8x8_P1_D8_n12.txt")
COUNTERS_UNEVEN = os.path.join(ROOT, "profiles", "counters_uneven16_D10group.txt")
COUNTERS_B32 = os.path.join(ROOT, "profiles", "counters_box32x16x16_P0_D12_n16_two_level.txt")
COUNTERS_B32_ASM = os.path.join(ROOT, "profiles", "counters_box32x16x16_P0_D12_n16_assembly_bytes.txt")


def measured_traffic(label, path=COUNTERS, field="bytes"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 byte counters
    (FETCH_SIZE / WRITE_SIZE scaled by a plain-copy calibration), or their ratio to
    the algorithmic bytes (field="ratio"), or None when the kernel's source file
    changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("kernel="):
            continue
        kv = dict(tok.split("=", 1) for tok in line.split())
        if kv["kernel"] != label:
            continue
        src = os.path.join(ROOT, kv["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["sha256"]:
            return None
        return float(kv[field])
    return None


# --------------------------------------------------------------------------- GPU path


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (--gpus {args.gpus} requested); sharding the assembly "
              "and solve over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        return copy_calib()
    if args.workload == "box32-batched":
        return main_box32(args)
    if args.workload == "uneven":
        return main_uneven(args)
    if args.workload == "box32-adjoint":
        return main_box32_adjoint(args)
    return main_box8(args)


def copy_calib():
    """A plain elementwise kernel reading and writing 1 GiB each, for calibrating
    the HBM byte counters."""
    import torch
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 5,
                      "kernel": "elementwise mul"}))


def main_box8(args):
    """The 3072-tet box (8x8x8 Kuhn cells, jitter 0.15h, P1 x Legendre D = 8, n = 12,
    mu = 0.05, walls R = 0.9, Gaussian patch source on x = 0).  One step = mesh
    build -> assembly -> source -> plain FP64 GMRES, FP32 GMRES corrections in FP64
    refinement, and the two-level solve, each to relative residual 1e-8."""
    import numpy as np

    import synth
    prob = synth.problem_c2()
    rule = 1 if args.rule == "seam" else 0
    base = None
    if not args.no_cpu_baseline and not args.kernels_only:
        base = cpu_baseline(prob, rule, args.cpu_tets)
        base["product_ms"], ms_sub, nt_sub = oracle_product_ms(synth.problem_c2(n_cells=4), 135, prob.nt)
        base["product_sample"] = (f"oracle CSR product on the same recipe with 4x4x4 cells ({nt_sub} tets, K = 135, "
                                  f"random blocks) {ms_sub:.1f} ms, one thread, scaled by tets to {prob.nt}")
        print(f"bench: cpu baseline {base['value']:.2f} blocks/s, product {base['product_ms']:.0f} ms",
              file=sys.stderr, flush=True)

    import torch

    from paper_1608_04607_amd import dfm

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    verts = torch.tensor(prob.verts, device=dev)
    tets = torch.tensor(prob.tets, device=dev)
    refl = torch.tensor(prob.refl, device=dev)
    mu = torch.tensor(prob.mu, device=dev)
    src = (0.0, 0.5, 0.5, 0.1)
    torch.cuda.synchronize()
    if args.kernels_only:
        mesh = dfm.Mesh(verts, tets, refl=refl)
        op = dfm.Operator(mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
        x = torch.rand(op.ndof, dtype=torch.float64, device=dev)
        for _ in range(5):
            op.apply(x)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "nodes": op.nodes, "K": op.K, "ndof": op.ndof,
                          "B_bytes": op.nbytes}))
        return

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def step(record):
        e = [ev() for _ in range(7)]
        e[0].record(stream)
        mesh = dfm.Mesh(verts, tets, refl=refl)
        e[1].record(stream)
        op = dfm.Operator(mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
        e[2].record(stream)
        rho0 = op.source_plane(0, 0.0, profile=1, params=src)
        e[3].record(stream)
        # plain FP64 GMRES, then FP32 GMRES corrections inside FP64 iterative refinement
        rho, info = op.solve(rho0, method="gmres", rtol=1e-8, restart=args.restart, max_iter=20000)
        e[4].record(stream)
        rho_m, info_m = op.solve(rho0, method="gmres", rtol=1e-8, restart=args.restart, max_iter=20000,
                                 precision=1)
        e[5].record(stream)
        # two-level sweeps (FP16 products on the matrix cores) inside FP64 refinement
        rho_t, info_t = op.solve(rho0, method="twolevel", rtol=1e-8, max_iter=20000)
        e[6].record(stream)
        if record is not None:
            diff = float(((rho_m - rho).norm() / rho.norm()).item())
            diff_t = float(((rho_t - rho).norm() / rho.norm()).item())
            record.append((e, info + info_m + [info_t[0]], op.nodes, op.nblocks, op.K, op.ndof, diff, diff_t))
        op.close()
        mesh.close()
        return rho

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    phase = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(6)] for r in recs])  # ms
    t_mesh, t_asm, t_src, t_solve, t_mixed, t_two = phase.mean(axis=0)
    info, info_m, info_t = recs[-1][1]
    nodes, nblocks, K, ndof, diff, diff_t = recs[-1][2:]
    blocks_per_s = nblocks * args.steps / (phase[:, 1].sum() / 1e3)

    # SpMV kernel: one dfm_apply launch per call, timed with events on the same stream
    op_mesh = dfm.Mesh(verts, tets, refl=refl)
    op = dfm.Operator(op_mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
    x = torch.rand(ndof, dtype=torch.float64, device=dev)
    for _ in range(3):
        op.apply(x)
    e0, e1 = ev(), ev()
    nrep = 20
    e0.record(stream)
    for _ in range(nrep):
        op.apply(x)
    e1.record(stream)
    torch.cuda.synchronize()
    t_spmv = e0.elapsed_time(e1) / nrep
    op.close()
    # FP32 assembly (dtype 1) of the same operator, for the precision comparison
    t32 = []
    for i in range(args.steps + 1):
        e0, e1 = ev(), ev()
        e0.record(stream)
        op32 = dfm.Operator(op_mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule,
                            dtype=1)
        e1.record(stream)
        torch.cuda.synchronize()
        if i:
            t32.append(e0.elapsed_time(e1))
        op32.close()
    op_mesh.close()
    t_asm32 = sum(t32) / len(t32)

    flops_asm = 2.0 * nodes * K * K
    asm_tflops = flops_asm / (t_asm / 1e3) / 1e12
    spmv_bytes = 8.0 * (12 * (ndof // (4 * K)) * K * K + 2 * ndof)
    spmv_gbs = spmv_bytes / (t_spmv / 1e3) / 1e9
    t_spmv_step = t_spmv * info[0]  # FP64 solve's operator applications
    asm_traffic = measured_traffic("k_assemble")
    roof_asm = {"kernel": "k_assemble", "bound": "mfma", "achieved": asm_tflops, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": asm_tflops / FP64_PEAK_TFLOPS, "traffic": asm_traffic,
                "algorithmic": f"2*Q*K^2 flop per block, Q summed over blocks = {nodes}, K = {K}",
                "hbm_GBs": None if asm_traffic is None else asm_traffic / (t_asm / 1e3) / 1e9,
                "hbm_frac": None if asm_traffic is None else asm_traffic / (t_asm / 1e3) / 1e9 / HBM_PEAK_GBS}
    roof_spmv = {"kernel": "k_spmv", "bound": "hbm", "achieved": spmv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": spmv_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("k_spmv_f64"),
                 "algorithmic": "8*(12*N*K^2 + 2*ndof) bytes per launch (B once, x and y once)"}
    dominant, other = (roof_asm, roof_spmv) if t_asm >= t_spmv_step else (roof_spmv, roof_asm)
    out = {
        "metric": METRIC,
        "value": blocks_per_s,
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"box8x8x8-kuhn-3072tets-jitter0.15_P1xLegendreD8_n12_{args.rule}-rule"
                               "_mu0.05_R0.9_gauss-patch_gmres1e-8",
                   "tets": int(prob.nt), "blocks": int(nblocks), "K": int(K), "ndof": int(ndof),
                   "quadrature_directions": int(nodes)},
        "phase_ms": {"mesh_build": t_mesh, "assemble": t_asm, "source": t_src, "solve_fp64": t_solve,
                     "solve_fp32_refined": t_mixed, "solve_twolevel": t_two},
        "solve_ms_per_rhs": min(t_mixed, t_two),
        "solve_precision": "fastest of: fp32 GMRES corrections, fp64 refinement residuals (solve_fp32_refined); "
                           "two-level sweeps with fp16 products, fp64 refinement residuals (solve_twolevel)",
        "solve_relres": info_m[2],
        "solve_iters": info_m[0],
        "solve_twolevel_ms_per_rhs": t_two,
        "solve_twolevel_relres": info_t[2],
        "solve_twolevel_sweeps": info_t[0],
        "solve_twolevel_rel_diff_vs_fp64": diff_t,
        "solve_twolevel_speedup_vs_fp64": t_solve / t_two,
        "solve_fp64_ms_per_rhs": t_solve,
        "solve_fp64_iters": info[0],
        "solve_fp64_relres": info[2],
        "solve_speedup_vs_fp64": t_solve / min(t_mixed, t_two),
        "solve_rel_diff_vs_fp64": diff,
        "spmv_ms": t_spmv,
        "assemble_fp32_ms": t_asm32,
        "assemble_fp32_blocks_per_s": nblocks / (t_asm32 / 1e3),
        "assemble_fp32_tflops": flops_asm / (t_asm32 / 1e3) / 1e12,
        "roofline": dominant,
        "roofline_other": other,
        "cpu_baseline": base,
    }
    if base is not None:
        # the oracle's solve: its product time times the plain FP64 solve's products
        base["solve_ms_per_rhs"] = base["product_ms"] * info[0]
        base["solve_sample"] = (f"oracle product time x the {info[0]} operator applications of the plain FP64 "
                                "GMRES solve of this run")
    print(json.dumps(out))


def main_box32(args):
    """The batched 49152-tet box (the default workload; see the module docstring).
    One step = mesh build -> FP64 assembly -> 128 point sources -> two-level solve
    of all 128 to relative residual 1e-8.  The per-rhs reference (one plain FP64
    Neumann solve), the batched FP64 product and true residuals are measured once,
    after the timed steps, on the last step's operator."""
    import numpy as np

    import synth
    prob = synth.problem_c3(nsrc=128)
    rule = 1 if args.rule == "seam" else 0
    base = None
    if not args.no_cpu_baseline and not args.kernels_only:
        base = cpu_baseline(prob, rule, min(args.cpu_tets, 8), "49152-tet box")
        base["product_ms"], ms_sub, nt_sub = oracle_product_ms(synth.problem_c3(cells=(8, 4, 4), nsrc=1), 91, prob.nt)
        base["product_sample"] = (f"oracle CSR product on the same recipe with 8x4x4 cells ({nt_sub} tets, K = 91, "
                                  f"random blocks) {ms_sub:.1f} ms, one thread, scaled by tets to {prob.nt}")
        print(f"bench: cpu baseline {base['value']:.2f} blocks/s, product {base['product_ms']:.0f} ms",
              file=sys.stderr, flush=True)

    import torch

    from paper_1608_04607_amd import dfm

    os.environ.setdefault("DFM_VERBOSE", "1")      # one stderr line per refinement stage
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    T = lambda a: torch.tensor(a, device=dev)  # noqa: E731
    verts, tets, refl, mu, xyz = T(prob.verts), T(prob.tets), T(prob.refl), T(prob.mu), T(prob.source["xyz"])
    R = int(xyz.shape[0])
    if args.kernels_only:
        mesh = dfm.Mesh(verts, tets, refl=refl)
        op = dfm.Operator(mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
        rho0 = op.source_points(xyz)
        op.solve(rho0, method="twolevel", rtol=1e-8, max_iter=int(os.environ.get("BENCH_PRODUCTS", "40")),
                 raise_nonconv=False)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "workload": "box32", "nodes": op.nodes, "K": op.K, "ndof": op.ndof,
                          "B_bytes": op.nbytes, "nrhs": R}))
        return
    torch.cuda.synchronize()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def step(record, keep=False):
        e = [ev() for _ in range(5)]
        e[0].record(stream)
        mesh = dfm.Mesh(verts, tets, refl=refl)
        e[1].record(stream)
        op = dfm.Operator(mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
        e[2].record(stream)
        rho0 = op.source_points(xyz)
        e[3].record(stream)
        op.product_timing(1)
        rho, info = op.solve(rho0, method="twolevel", rtol=1e-8, max_iter=20000)
        e[4].record(stream)
        timing = op.product_timing(0)
        if record is not None:
            record.append((e, info, timing))
        print(f"bench: step done, {info[0][0]} products, worst relres {max(i[2] for i in info):.2e}",
              file=sys.stderr, flush=True)
        if keep:
            return mesh, op, rho0, rho, info
        del rho, rho0
        op.close()
        mesh.close()
        return None

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        kept = step(recs, keep=i == args.steps - 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mesh, op, rho0, rho, info = kept

    phase = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(4)] for r in recs])  # ms
    t_mesh, t_asm, t_src, t_solve = phase.mean(axis=0)
    blocks, K, nodes, ndof = op.nblocks, op.K, op.nodes, op.ndof
    prod_ms = sum(r[2][0] for r in recs)
    prod_launches = sum(r[2][1] for r in recs)
    prod_bytes = sum(r[2][2] for r in recs)
    launch_ms = prod_ms / prod_launches
    spmm_gbs = prod_bytes / (prod_ms / 1e3) / 1e9
    flops_asm = 2.0 * nodes * K * K
    asm_tf = flops_asm / (t_asm / 1e3) / 1e12
    roof_spmm = {"kernel": "k_spmm16_lds", "bound": "hbm", "achieved": spmm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": spmm_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("k_spmm16_lds", COUNTERS_B32),
                 "avg_launch_ms": launch_ms, "launches": prod_launches,
                 "algorithmic_bytes_per_launch": prod_bytes / prod_launches,
                 "algorithmic": "per tet of a launch (one colour): 4 block rows x (3 ceil(K/32) slot chunks + "
                                "3 correction chunks) x K x 32 x 2 B of FP16 B, 4 x nrhs x Kp8 x 2 B of x read, "
                                "as much of y written, 4 x F x nrhs x 4 B of coarse projections (K = 91, Kp8 = 96, "
                                "F = 9, nrhs = 128)",
                 "timed": "every product launch of the timed steps' solves, HIP events on the solve's stream"}
    roof_asm = {"kernel": "k_assemble", "bound": "mfma", "achieved": asm_tf, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": asm_tf / FP64_PEAK_TFLOPS,
                "traffic": measured_traffic("k_assemble", COUNTERS_B32_ASM),
                "algorithmic": f"2*Q*K^2 flop per launch, Q = {nodes} directions summed over blocks, K = {K}",
                "timed": "the assembly phase of each timed step (HIP events)"}
    t_spmm_step = prod_ms / len(recs)
    dominant, other = (roof_spmm, roof_asm) if t_spmm_step >= t_asm else (roof_asm, roof_spmm)

    # true FP64 residuals of three of the last step's solutions
    worst = 0.0
    for r in (0, R // 2, R - 1):
        res = rho0[r] - (rho[r] - op.apply(rho[r]))
        worst = max(worst, float((res.norm() / rho0[r].norm()).item()))
    # the batched FP64 product (dfm_residual: every block row read once per 128
    # right-hand sides on the FP64 matrix cores, FP64 accumulation) over all R
    op.residual(rho0, rho)
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(2):
        res = op.residual(rho0, rho)
    e1.record(stream)
    torch.cuda.synchronize()
    t_res = e0.elapsed_time(e1) / 2
    del res
    out = {
        "metric": METRIC,
        "value": blocks / (t_asm / 1e3),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 assembly; f16 products with f32 accumulation in the solve, f64 residuals",
        "data": "synthetic",
        "config": {"workload": "box32x16x16-kuhn-49152tets-jitter0.1_P0xLegendreD12_n16_"
                               f"{args.rule}-rule_mu-lognormal(ln0.02,0.5)_R0.9_128-point-sources_batched-1e-8",
                   "tets": int(prob.nt), "blocks": int(blocks), "K": int(K), "ndof": int(ndof), "nrhs": R,
                   "quadrature_directions": int(nodes)},
        "phase_ms": {"mesh_build": t_mesh, "assemble": t_asm, "sources": t_src, "solve_128rhs": t_solve},
        "step_ms_per_rhs": wall * 1e3 / args.steps / R,
        "solve_ms_per_rhs": t_solve / R,
        "solve_method": "two-level: coloured Gauss-Seidel sweeps with a coarse correction, FP16 products on the "
                        "matrix cores, FP64 refinement residuals",
        "solve_products": int(info[0][0]),
        "solve_relres_worst": max(i[2] for i in info),
        "solve_true_relres_sampled": worst,
        "product_ms_per_step": t_spmm_step,
        "fp64_batched_product_ms": t_res,
        "roofline": dominant,
        "roofline_other": other,
        "cpu_baseline": base,
    }
    if not args.no_fp64_reference:
        print("bench: plain FP64 single-rhs Neumann reference", file=sys.stderr, flush=True)
        e0, e1 = ev(), ev()
        e0.record(stream)
        rho64, info64 = op.solve(rho0[0], method="neumann", rtol=1e-8, max_iter=40000)
        e1.record(stream)
        torch.cuda.synchronize()
        t64 = e0.elapsed_time(e1)
        n64 = int(info64[0][0])
        out.update({
            "fp64_ms_per_rhs": t64, "fp64_method": "plain FP64 Neumann, one rhs", "fp64_products": n64,
            "fp64_relres": info64[0][2],
            "speedup_per_rhs_vs_fp64": t64 / (t_solve / R),
            "rel_diff_vs_fp64_rhs0": float(((rho[0] - rho64).norm() / rho64.norm()).item()),
            "fp64_batched_ms_per_rhs_est": t_res * n64 / R,
            "speedup_per_rhs_vs_fp64_batched_est": t_res * n64 / t_solve,
            "fp64_batched_note": "plain FP64 Neumann over all 128 at once, estimated as the measured batched FP64 "
                                 "product (dfm_residual) x the plain solve's products / 128: "
                                 "fp64_ms_per_rhs / this is the gain of batching alone, this / solve_ms_per_rhs "
                                 "that of the method and precision",
        })
        if base is not None:
            base["solve_ms_per_rhs"] = base["product_ms"] * n64
            base["solve_sample"] = (f"oracle product time x the {n64} products of the plain FP64 Neumann solve of "
                                    "this run")
        del rho64
    del rho, rho0
    op.close()
    mesh.close()
    print(json.dumps(out))


def main_uneven(args):
    """Uneven batch of independent instances: 256 boxes (1, U[1,4], U[1,4]) with a
    log-uniform target of 500-20000 tets (384-20412 once the cells are rounded), jitter 0.2h, mu ~ U[0, 0.1] per box, R = 0.9, P0 x
    Legendre of degree uniform in {4,6,8,10} with n = D + 4, 4 isotropic point
    sources per box.  Instances of one degree form one mesh (block-diagonal B,
    assembled in FP32 by one launch); one step = for every group: mesh build ->
    FP32 assembly -> sources -> two-level solve of the group's instances (coloured
    sweeps with a coarse correction per instance, FP16 products of the 4 right-hand
    sides, FP64 residuals of the FP32-stored operator) until every instance's own
    relative residual is <= 1e-8 -> release.  Warmup runs the same on the first 8 boxes.  The plain FP64 reference
    solves a few boxes per degree one by one (FP64 assembly, FP64 Neumann per
    source); its whole-batch time is extrapolated per degree by tet count.
    `value` is assembly blocks/s over all groups."""
    import numpy as np

    import synth
    probs = synth.problem_c5(n_instances=args.instances)
    rule = 1 if args.rule == "seam" else 0
    degrees = sorted({p.mom_degree for p in probs})
    base = None
    if not args.no_cpu_baseline:
        # the oracle on one tet per core of the first box of every degree, combined
        # with the workload's own mix of blocks per degree
        blocks_by_d = {d: 12 * sum(p.nt for p in probs if p.mom_degree == d) for d in degrees}
        t_est, parts, cores = 0.0, [], 0
        per = min(16, len(os.sched_getaffinity(0)))
        for d in degrees:
            p = next(p for p in probs if p.mom_degree == d)
            b, dt, cores = _oracle_blocks(p, rule, per)
            t_est += blocks_by_d[d] * dt / b
            parts.append(f"D{d}: {b} blocks in {dt:.1f} s")
        base = {"value": sum(blocks_by_d.values()) / t_est, "unit": "blocks/s", "cores": cores, "kind": "oracle",
                "sample": f"{per} tets (seed 6) of the first box of every degree, FP64 NumPy oracle, "
                          f"{cores} worker processes ({'; '.join(parts)}), weighted by the batch's blocks "
                          "per degree"}
        print(f"bench: cpu baseline {base['value']:.2f} blocks/s", file=sys.stderr, flush=True)

    import torch

    from paper_1608_04607_amd import dfm
    from paper_1608_04607_amd.batch import UnevenBatch

    stream = torch.cuda.current_stream()

    def ev_new():
        return torch.cuda.Event(enable_timing=True)

    if args.kernels_only:
        # FP32 assembly of every degree group (released after it), then the largest
        # group again and five 4-rhs streaming products
        batch = UnevenBatch(probs, rule=rule, dtype=1)
        for g in batch.groups:
            batch.assemble(g)
            torch.cuda.synchronize()
            print(f"bench: assembled D={g.key[2]} ({g.mesh.nt} tets, {g.op.nodes} directions, K = {g.op.K})",
                  file=sys.stderr, flush=True)
            batch.release(g)
        g = max(batch.groups, key=lambda g: g.tet_offsets[-1] * (g.key[2] + 1) ** 4)
        batch.assemble(g)
        x32 = g.rho0.float()
        for _ in range(5):
            g.op.apply_f32(x32)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "workload": f"uneven-{len(probs)}", "degree": g.key[2],
                          "boxes": len(g.members), "tets": g.mesh.nt, "K": g.op.K, "nrhs": g.nsrc,
                          "B_bytes": g.op.nbytes, "product_bytes": g.op.nbytes + 16.0 * g.nsrc * g.op.ndof}))
        return

    class TimedBatch(UnevenBatch):
        """Turns on the event timing of the FP16 product launches of each group's
        solves as soon as the group's operator exists."""

        def assemble(self, g, stream=None):
            super().assemble(g, stream=stream)
            g.op.product_timing(1)

    def run(batch, label):
        """Every group once (with --overlap the next group is assembled beside the solve of
        this one); per group (mesh+assembly, sources, solve) ms and stats."""
        rows = []

        def progress(g, worst):
            print(f"bench: {label} D={g.key[2]} ({len(g.members)} boxes, {g.mesh.nt} tets): "
                  f"{g.products} batched products, worst box relres {worst:.2e}", file=sys.stderr, flush=True)

        def on_group(g, t_solve):
            ev = g.events
            pt_ms, pt_n, pt_b = g.op.product_timing(0)
            rows.append({"degree": g.key[2], "boxes": len(g.members), "tets": g.mesh.nt, "K": g.op.K,
                         "product16_ms": pt_ms, "product16_launches": pt_n, "product16_bytes": pt_b,
                         "blocks": g.op.nblocks, "nodes": g.op.nodes, "B_bytes": g.op.nbytes, "nrhs": g.nsrc,
                         "ms_assemble": ev[0].elapsed_time(ev[1]), "ms_sources": ev[1].elapsed_time(ev[2]),
                         "ms_solve": t_solve, "products": g.products,
                         "work_fraction": sum(mp * (g.tet_offsets[m + 1] - g.tet_offsets[m])
                                              for m, mp in enumerate(g.member_products)) / (g.products * g.mesh.nt),
                         "worst_member_relres": max(max(r) for r in g.relres)})
            if label == "step":
                # the streaming FP32 product alone, 4 right-hand sides (HIP events on this
                # stream); the next group's assembly has finished by now
                x32 = g.rho.float()
                g.op.apply_f32(x32)
                e0, e1 = ev_new(), ev_new()
                e0.record(stream)
                for _ in range(5):
                    g.op.apply_f32(x32)
                e1.record(stream)
                torch.cuda.synchronize()
                rows[-1]["ms_product"] = e0.elapsed_time(e1) / 5
                del x32
                rows[-1]["rho"] = [batch.solution(i).clone() for i in g.members[:args.fp64_sample]]

        batch.solve_all(rtol=1e-8, overlap=args.overlap, progress=progress, on_group=on_group)
        return rows

    for _ in range(args.warmup):
        run(TimedBatch(probs[:8], rule=rule, dtype=1), "warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch = TimedBatch(probs, rule=rule, dtype=1)
        rows = run(batch, "step")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # plain FP64 reference: the first boxes of every degree, one by one
    T = lambda a: torch.tensor(a, device="cuda:0")  # noqa: E731
    ref = {}
    worst_diff = 0.0
    for gi, g in enumerate(batch.groups):
        t_box, nt_box = 0.0, 0
        for m, i in enumerate(g.members[:args.fp64_sample]):
            p = probs[i]
            print(f"bench: plain FP64 reference, box {i} (D={p.mom_degree}, {p.nt} tets)", file=sys.stderr,
                  flush=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            mesh = dfm.Mesh(T(p.verts), T(p.tets), refl=T(p.refl))
            op = dfm.Operator(mesh, T(p.mu), p.pos_order, dfm.LEGENDRE, p.mom_degree, p.quad_n, rule=rule)
            rho0 = op.source_points(T(p.source["xyz"]))
            rho, _ = op.solve(rho0, method="neumann", rtol=1e-8, max_iter=100000)
            torch.cuda.synchronize()
            t_box += (time.perf_counter() - t1) * 1e3
            nt_box += p.nt
            got = rows[gi]["rho"][m]
            worst_diff = max(worst_diff, float(((got - rho).norm() / rho.norm()).item()))
            op.close()
            mesh.close()
        ref[g.key[2]] = (t_box, nt_box, rows[gi]["tets"])
    t64_est = sum(t * nt_all / nt for t, nt, nt_all in ref.values())

    nblocks = sum(r["blocks"] for r in rows)
    t_asm = sum(r["ms_assemble"] for r in rows)
    t_src = sum(r["ms_sources"] for r in rows)
    t_solve = sum(r["ms_solve"] for r in rows)
    nrhs = sum(r["boxes"] * r["nrhs"] for r in rows)
    # the streaming product with every box multiplied, on the largest group
    pb = [r["B_bytes"] + 16.0 * r["nrhs"] * 4 * r["tets"] * r["K"] for r in rows]
    ib = max(range(len(rows)), key=lambda i: rows[i]["B_bytes"])
    big = rows[ib]
    prod_bytes, prod_ms = pb[ib], big["ms_product"]
    prod_gbs = prod_bytes / (prod_ms / 1e3) / 1e9
    flops_asm = sum(2.0 * r["nodes"] * r["K"] ** 2 for r in rows)
    for r in rows:
        r.pop("rho", None)
    # the two rooflines of the step: the FP32 assembly (matrix cores) and the FP16
    # product of the group solves (HBM), timed with events inside the library
    asm_tf = flops_asm / (t_asm / 1e3) / 1e12
    roof_asm = {"kernel": "k_assemble (dtype 1)", "bound": "mfma", "achieved": asm_tf, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": asm_tf / FP32_PEAK_TFLOPS, "traffic": None,
                "algorithmic": "2*Q*K^2 flop per group launch, summed over the four degree groups",
                "timed": "the mesh build + assembly events of every group (basis rows FP32, node geometry FP64)"}
    p16_ms = sum(r["product16_ms"] for r in rows)
    p16_n = sum(r["product16_launches"] for r in rows)
    p16_b = sum(r["product16_bytes"] for r in rows)
    p16_gbs = p16_b / (p16_ms / 1e3) / 1e9 if p16_ms > 0 else 0.0
    roof_p16 = {"kernel": "k_spmm16", "bound": "hbm", "achieved": p16_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": p16_gbs / HBM_PEAK_GBS, "traffic": None, "launches": p16_n,
                "avg_launch_ms": p16_ms / max(p16_n, 1),
                "algorithmic": "per tet of a launch: its 4 block rows of FP16 B (slot and correction chunks), "
                               "x read and y written once for the 4 rhs, d0 (dfm_product_timing)",
                "timed": "every product launch of the step's group solves, HIP events on the solve's stream"}
    out = {
        "metric": METRIC,
        "value": nblocks * args.steps / (t_asm / 1e3),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 basis rows, contraction and storage (f64 geometry, weights, Gram solve); f32 products, f64 residuals",
        "data": "synthetic",
        "config": {"workload": f"uneven-{len(probs)}-boxes-(1,U[1,4],U[1,4])-logU[500,20000]tets-jitter0.2"
                               f"_P0xLegendreD{{4,6,8,10}}_n=D+4_{args.rule}-rule_mu-U[0,0.1]_R0.9"
                               "_4-point-sources-each_batched-1e-8",
                   "boxes": len(probs), "tets": int(sum(r["tets"] for r in rows)), "blocks": int(nblocks),
                   "rhs": int(nrhs), "groups": [{k: v for k, v in r.items()} for r in rows]},
        "phase_ms": {"mesh_and_assemble": t_asm, "sources": t_src, "solve_batched": t_solve},
        "overlap": args.overlap,
        "assemble_tflops_fp32": flops_asm / (t_asm / 1e3) / 1e12,
        "solve_ms_per_rhs": t_solve / nrhs,
        "solve_precision": "two-level sweeps per degree group (FP16 products of 4 rhs, coarse correction per "
                           "instance), fp64 residuals of the fp32-stored B; every box's own relres <= 1e-8; "
                           "converged boxes leave the products",
        "solve_work_fraction": sum(r["work_fraction"] * r["products"] * r["tets"] for r in rows)
                               / sum(r["products"] * r["tets"] for r in rows),
        "solve_worst_member_relres": max(r["worst_member_relres"] for r in rows),
        "solve_fp64_ms_per_rhs_est": t64_est / nrhs,
        "solve_fp64_method": f"plain fp64, box by box: fp64 assembly + fp64 Neumann per source, {args.fp64_sample} "
                             "boxes per degree timed, scaled per degree by tets",
        "solve_fp64_sample_ms": {f"D{d}": v[0] for d, v in ref.items()},
        "speedup_vs_fp64_box_by_box_est": t64_est / (t_asm + t_src + t_solve),
        "rel_diff_vs_fp64_sampled": worst_diff,
        "roofline": roof_asm if t_asm >= p16_ms else roof_p16,
        "roofline_other": roof_p16 if t_asm >= p16_ms else roof_asm,
        "streaming_product_fp32": {"kernel": "k_spmv_rhs<4>", "bound": "hbm", "achieved": prod_gbs,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": prod_gbs / HBM_PEAK_GBS,
                                   "note": "the FP32 Neumann product of method 0 (not used by this step's solve), "
                                           "five launches on the largest group with every box multiplied",
                                   "algorithmic": f"B32 bytes + 16*R*ndof per launch, R = 4: {prod_bytes:.3e} B",
                                   "ms_per_launch": prod_ms,
                                   "traffic_ratio_small_group": measured_traffic("k_spmv_rhs4", COUNTERS_UNEVEN,
                                                                                 "ratio")},
        "cpu_baseline": base,
    }
    print(json.dumps(out))


def gradient_check_c4(prob, mesh, op, mu, xyz, src, rho, dmu, dw, box, rule, dfm, torch, nparam=32, seed=4,
                      h=1e-6):
    """Check of the adjoint gradients on the full 49152-tet box.

    Source weights: J is linear in w, so dJ/dw_s = g . rho_s exactly, with rho_s the
    solution for source s alone -- all 64 from one batched two-level solve.

    Damping: `nparam` parameters drawn uniformly (seed 4) from the 49152 mu_e and
    the 64 w_s.  A central difference of J itself in mu_e is limited by
    cancellation (J changes by ~1e-9 of itself for a step of 1e-6), so the
    difference is taken where it is exact to first order: J(mu) = g(mu) . (I -
    B(mu))^-1 rho0 gives
        dJ/dmu_e = g . (I - B)^-1 [(dB/dmu_e) rho] + (dg/dmu_e) . rho,
    and dB/dmu_e, dg/dmu_e (nonzero only in tet e's 12 blocks and 4 slots) are
    replaced by central differences of the blocks and of g assembled with mu_e +- h
    (on the tet and its face neighbours, the same frames as in the full mesh).  The
    difference quotients with steps h and 2h are both formed (their spread is the
    difference's own error) and all tangent systems are solved in one batched
    two-level solve.  w-type draws use the exact linear check."""
    import numpy as np
    dev = rho.device
    K = op.K
    nt = prob.nt
    R = src.shape[0]
    out = {}
    # 1. all source weights
    os.environ.setdefault("DFM_VERBOSE", "1")      # one stderr line per refinement stage
    print("bench: gradient check: batched solve of the 64 unit sources", file=sys.stderr, flush=True)
    rho_s, info = op.solve(src, method="twolevel", rtol=1e-10, max_iter=20000)
    Js = op.receiver_energy(rho_s, box)
    dw_h, Js_h = dw.cpu().numpy(), Js.cpu().numpy()
    out["w_all"] = {"count": int(R), "max_rel_diff": float(np.abs(dw_h - Js_h).max() / np.abs(Js_h).max()),
                    "method": "dJ/dw_s = g . rho_s, rho_s from one batched two-level solve to 1e-10",
                    "products": int(info[0][0])}
    del rho_s
    # 2. random parameters
    draws = np.random.default_rng(seed).choice(nt + R, nparam, replace=False)
    nbr = mesh.export()[0].cpu().numpy()
    blocks_e, dest_e = op.export_tets(torch.tensor([int(d) for d in draws if d < nt] or [0], device=dev))
    dest_map = {int(d): dest_e[i].cpu().numpy() for i, d in enumerate([d for d in draws if d < nt])}
    tets_all = prob.tets
    verts_t = torch.tensor(prob.verts, device=dev)
    rhs, meta = [], []
    rho_h = rho
    for d in draws:
        d = int(d)
        if d >= nt:
            meta.append(("w", d - nt))
            continue
        print(f"bench: gradient check: central differences of the blocks of tet {d}", file=sys.stderr, flush=True)
        sub = [d] + sorted({int(x) // 4 for x in nbr[d] if x >= 0})
        msub = dfm.Mesh(verts_t, torch.tensor(tets_all[sub], device=dev), refl=torch.tensor(prob.refl[sub], device=dev))
        parts = {}
        for step in (h, 2 * h):
            for sgn in (1.0, -1.0):
                mu_sub = mu[sub].clone()
                mu_sub[0] += sgn * step
                osub = dfm.Operator(msub, mu_sub, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n,
                                    rule=rule)
                bl, _ = osub.export_tets(torch.tensor([0], device=dev))
                g_sub = osub.receiver_functional(box)[: 4 * K]
                parts[(step, sgn)] = (bl[0], g_sub)
                osub.close()
        msub.close()
        for step in (h, 2 * h):
            dB = (parts[(step, 1.0)][0] - parts[(step, -1.0)][0]) / (2 * step)     # [4][3][K][K]
            dg = (parts[(step, 1.0)][1] - parts[(step, -1.0)][1]) / (2 * step)     # [4 K]
            r = torch.zeros(op.ndof, dtype=torch.float64, device=dev)
            for lo in range(4):
                dst = int(dest_map[d][lo])
                for s_ in range(3):
                    li = s_ if s_ < lo else s_ + 1
                    r[dst * K:(dst + 1) * K] += dB[lo, s_] @ rho_h[(4 * d + li) * K:(4 * d + li + 1) * K]
            rhs.append(r)
            meta.append(("mu", d, step, float(dg @ rho_h[4 * d * K:(4 * d + 4) * K])))
    tau, tinfo = op.solve(torch.stack(rhs), method="twolevel", rtol=1e-10, max_iter=20000)
    gt = op.receiver_energy(tau, box).cpu().numpy()
    dmu_h = dmu.cpu().numpy()
    rows, k = [], 0
    for m in meta:
        if m[0] == "w":
            rows.append({"param": f"w[{m[1]}]", "adjoint": float(dw_h[m[1]]), "fd": float(Js_h[m[1]]),
                         "rel_diff": float(abs(dw_h[m[1]] - Js_h[m[1]]) / abs(Js_h[m[1]]))})
            continue
        if m[2] != h:
            continue
        fd_h = gt[k] + m[3]
        fd_2h = gt[k + 1] + meta[meta.index(m) + 1][3]
        k += 2
        e = m[1]
        scale = max(abs(dmu_h[e]), 1e-300)
        rows.append({"param": f"mu[{e}]", "adjoint": float(dmu_h[e]), "fd": float(fd_h),
                     "rel_diff": float(abs(fd_h - dmu_h[e]) / scale),
                     "fd_h_vs_2h": float(abs(fd_h - fd_2h) / scale)})
    gmax = float(np.abs(dmu_h).max())
    out["params"] = rows
    out["count"] = len(rows)
    out["max_rel_diff"] = max(r["rel_diff"] for r in rows)
    out["max_abs_diff_over_max_gradient"] = max(abs(r["fd"] - r["adjoint"]) for r in rows if r["param"][0] == "m") / gmax
    out["fd_own_error_max"] = max(r.get("fd_h_vs_2h", 0.0) for r in rows)
    out["method"] = ("central differences (steps 1e-6 and 2e-6) of the blocks and of g of the perturbed tet, "
                     "through one batched two-level solve of the tangent systems to 1e-10")
    out["tangent_products"] = int(tinfo[0][0])
    return out


def main_box32_adjoint(args):
    """Receiver-energy gradients on the 49152-tet box: J = energy in [1.6,1.9] x
    [0.4,0.6]^2 of the stationary density for rho0 = sum_s w_s src_s over the first
    64 of the 128 point sources (w_s = 1).  One step = FP64 assembly -> 64 sources
    -> forward GMRES(100) to 1e-10 -> receiver functional -> adjoint (transposed
    GMRES(100) to 1e-10, dB/dmu contraction, dJ/dw = lambda . src_s), both solves
    with FP32 corrections inside FP64 refinement.  After the timed steps: the same
    two solves in plain FP64 (time and gradient difference), duality g.rho =
    lambda.rho0, and the gradient check of gradient_check_c4.  `value` is assembly
    blocks/s."""
    import numpy as np

    import synth
    prob = synth.problem_c3(nsrc=128)
    import torch

    from paper_1608_04607_amd import dfm

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    T = lambda a: torch.tensor(a, device=dev)  # noqa: E731
    verts, tets, refl, mu = T(prob.verts), T(prob.tets), T(prob.refl), T(prob.mu)
    xyz = T(prob.source["xyz"][:64])
    box = (1.6, 1.9, 0.4, 0.6, 0.4, 0.6)
    rule = 1 if args.rule == "seam" else 0
    mesh = dfm.Mesh(verts, tets, refl=refl)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def forward(mu_, rtol):
        op = dfm.Operator(mesh, mu_, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
        src = op.source_points(xyz)
        rho0 = src.sum(0)
        rho, info = op.solve(rho0, method="gmres", rtol=rtol, restart=100, max_iter=40000)
        g = op.receiver_functional(box)
        return op, src, rho0, rho, g, info

    recs = []
    t0 = time.perf_counter()
    for i in range(args.warmup + args.steps):
        if i == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        e = [ev() for _ in range(5)]
        e[0].record(stream)
        op = dfm.Operator(mesh, mu, prob.pos_order, dfm.LEGENDRE, prob.mom_degree, prob.quad_n, rule=rule)
        e[1].record(stream)
        src = op.source_points(xyz)
        rho0 = src.sum(0)
        rho, info = op.solve(rho0, method="gmres", rtol=1e-10, restart=100, max_iter=40000, precision=1)
        e[2].record(stream)
        g = op.receiver_functional(box)
        J = float((g * rho).sum())
        e[3].record(stream)
        lam, dmu, dw, ainfo = op.adjoint(rho, box, src=src, rtol=1e-10, restart=100, max_iter=40000, precision=1)
        e[4].record(stream)
        torch.cuda.synchronize()
        print(f"bench: step {i}: forward {info[0][0]} iterations, adjoint {ainfo[0]} iterations", file=sys.stderr,
              flush=True)
        if i >= args.warmup:
            recs.append([e[k].elapsed_time(e[k + 1]) for k in range(4)])
        if i < args.warmup + args.steps - 1:
            op.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_asm, t_fwd, t_g, t_adj = np.array(recs).mean(axis=0)
    duality = abs(J - float((lam * rho0).sum())) / abs(J)
    dmu_h = dmu.cpu().numpy()
    # plain FP64 forward and adjoint solves of the same step, for comparison
    print("bench: plain FP64 forward and adjoint solves", file=sys.stderr, flush=True)
    e = [ev() for _ in range(3)]
    e[0].record(stream)
    rho64, info64 = op.solve(rho0, method="gmres", rtol=1e-10, restart=100, max_iter=40000)
    e[1].record(stream)
    torch.cuda.synchronize()
    print(f"bench: plain FP64 forward {info64[0][0]} iterations", file=sys.stderr, flush=True)
    _, dmu64, dw64, ainfo64 = op.adjoint(rho64, box, src=src, rtol=1e-10, restart=100, max_iter=40000)
    e[2].record(stream)
    torch.cuda.synchronize()
    t_fwd64, t_adj64 = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    grad_diff = max(float((dmu - dmu64).abs().max() / dmu64.abs().max()),
                    float((dw - dw64).abs().max() / dw64.abs().max()))
    del rho64, dmu64, dw64
    e_max = int(np.abs(dmu_h).argmax())
    check = gradient_check_c4(prob, mesh, op, mu, xyz, src, rho, dmu, dw, box, rule, dfm, torch)
    op.close()
    del src, rho0, rho, lam
    torch.cuda.empty_cache()
    nblocks = 12 * prob.nt
    out = {
        "metric": METRIC,
        "value": nblocks / (t_asm / 1e3),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"box32x16x16-kuhn-49152tets-jitter0.1_P0xLegendreD12_n16_{args.rule}-rule"
                               "_mu-lognormal(ln0.02,0.5)_R0.9_64-point-sources_receiver[1.6,1.9]x[0.4,0.6]^2"
                               "_adjoint-gradients",
                   "tets": int(prob.nt), "blocks": int(nblocks), "sources": 64,
                   "gradient_sizes": {"d_mu": int(prob.nt), "d_w": 64}},
        "phase_ms": {"assemble": t_asm, "sources_and_forward_solve": t_fwd, "receiver_functional": t_g,
                     "adjoint": t_adj},
        "solve_precision": "fp32 GMRES(100) corrections inside fp64 refinement, forward and transposed, to 1e-10",
        "forward_iters": info[0][0],
        "adjoint_iters": ainfo[0],
        "adjoint_relres": ainfo[2],
        "fp64_forward_ms": t_fwd64,
        "fp64_adjoint_ms": t_adj64,
        "fp64_forward_iters": info64[0][0],
        "fp64_adjoint_iters": ainfo64[0],
        "speedup_vs_fp64": (t_fwd64 + t_adj64) / (t_fwd + t_adj),
        "gradient_rel_diff_vs_fp64": grad_diff,
        "J": J,
        "duality_rel_diff": duality,
        "gradient_check": check,
        "roofline": None,
        "cpu_baseline": None,
    }
    mesh.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
