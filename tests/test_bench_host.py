"""Host-side behaviour of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    """The path runs on one GPU; a request for more exits with status 2 and says why."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_bench_help_lists_the_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for w in ("box8", "box32-batched", "box32-adjoint", "uneven"):
        assert w in r.stdout


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_cpu_baseline_leg_times_the_oracle():
    """The bench's CPU leg runs the unmodified oracle in a worker pool and reports
    blocks/s, the cores used and what was sampled."""
    import numpy as np

    import synth
    bench = _bench()
    v, t = synth.kuhn_box((1, 1, 1), (1.0, 1.0, 1.0), jitter=0.1, seed=1)
    p = synth.Problem(name="tiny", verts=v, tets=t, mu=np.full(t.shape[0], 0.05), refl=np.full((t.shape[0], 4), 0.9),
                      pos_order=0, mom_degree=2, quad_n=4)
    out = bench.cpu_baseline(p, 1, 3, "one-cell test box")
    assert out["kind"] == "oracle" and out["unit"] == "blocks/s"
    assert out["value"] > 0 and 1 <= out["cores"] <= 16
    assert "3 tets (36 blocks)" in out["sample"]


def test_measured_traffic_needs_the_counted_source(tmp_path):
    """Byte counters are reported only while the kernel's source is the one counted."""
    import hashlib
    bench = _bench()
    src = "paper_1608_04607_amd/csrc/apply.hip"
    h = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
    f = tmp_path / "counters.txt"
    f.write_text(f"# test\nkernel=k source={src} sha256={h} bytes=123.0 ratio=1.5\n"
                 f"kernel=old source={src} sha256=0000000000000000 bytes=9.0 ratio=2.0\n")
    assert bench.measured_traffic("k", str(f)) == 123.0
    assert bench.measured_traffic("k", str(f), "ratio") == 1.5
    assert bench.measured_traffic("old", str(f)) is None
    assert bench.measured_traffic("missing", str(f)) is None


def test_oracle_product_leg_scales_by_tets():
    """The solve leg of the CPU baseline times the oracle's own sparse product on a
    sub-box and scales it to the full tet count; it reports the host's CPUs too."""
    import numpy as np

    import synth
    bench = _bench()
    sub = synth.problem_c3(cells=(2, 1, 1), nsrc=1)
    full_ms, sub_ms, nt_sub = bench.oracle_product_ms(sub, 6, 10 * sub.nt, min_s=0.05)
    assert nt_sub == sub.nt == 12
    assert sub_ms > 0 and np.isclose(full_ms, 10 * sub_ms)
    v, t = synth.kuhn_box((1, 1, 1), (1.0, 1.0, 1.0), jitter=0.1, seed=1)
    p = synth.Problem(name="tiny", verts=v, tets=t, mu=np.full(t.shape[0], 0.05), refl=np.full((t.shape[0], 4), 0.9),
                      pos_order=0, mom_degree=2, quad_n=4)
    out = bench.cpu_baseline(p, 1, 2, "one-cell test box")
    assert out["host_cpus"] == len(os.sched_getaffinity(0)) and out["cores"] <= out["host_cpus"]
