"""Host-side checks of bench.py's command line (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("l20", "l24", "l12", "batch", "serve", "gram", "slices"):
        assert w in r.stdout


def test_traffic_is_taken_only_from_matching_counter_files():
    sys.path.insert(0, ROOT)
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    # no counter file for this workload
    assert b.read_traffic("apply2", "l12", "f64") is None
    # counters of the mixed-precision L=24 workload do not describe an FP64 run of it
    assert b.read_traffic("apply2", "l24", "f64") is None
    # the committed files carry their workload and the source hash they were taken with
    for wl, prec in (("l20", "f64"), ("l24", "mixed")):
        txt = open(os.path.join(ROOT, "profiles", f"cg_apply_{wl}_counters.md")).read()
        assert f"counters_workload: {wl}" in txt and f"counters_precision: {prec}" in txt
        t = b.read_traffic("apply2", wl, prec)
        if f"apply_src_sha256_16: {b.apply_src_hash()}" in txt:
            assert t is not None and t > 0
        else:
            assert t is None


def test_cg_launch_widths_from_the_solve_counts():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    # the L=24 solve: 17,193 steps on 128 columns, 154,605 on the 64 wanted ones
    assert b.cg_launch_widths(171798, 12095424, 128, 64) == {128: 17193, 64: 154605}
    # no guard columns: every step on the whole block
    assert b.cg_launch_widths(1000, 64000, 64, 32) == {64: 1000}
    # counts that no mix of the two widths gives
    assert b.cg_launch_widths(1000, 64001, 64, 32) == {}
    assert b.cg_launch_widths(1000, 10, 64, 32) == {}
