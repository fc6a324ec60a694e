"""Host-side checks of the benchmark script (no GPU): it refuses more than
one GPU with a message, and its measured-traffic table is keyed to the
evaluation sources and launch shapes it reports."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_for_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_table_matches_sources_and_shapes():
    b = _bench_module()
    for prec in ("fp64", "mixed", "split"):
        t = b.MEASURED_TRAFFIC[prec]
        h = b.kernel_sources_hash(t["launch"]["j_source"])
        assert t["fetch_bytes"] > 0 and t["write_bytes"] > 0
        assert t["launch"]["j_source"] in b.JSOURCES
        # reported only for the profiled sources and shape
        if t["sources_sha256"] == h:
            assert b.measured_traffic(prec, t["launch"]) == t["fetch_bytes"] + t["write_bytes"]
        other = dict(t["launch"], j_split=t["launch"]["j_split"] + 1)
        assert b.measured_traffic(prec, other) is None


def test_peaks_and_flop_counts():
    b = _bench_module()
    # 256 CUs x 4 SIMD16 x 2 flops x 2.4 GHz (FP64); FP32 with packed issue twice that
    assert abs(b.PEAK_TFLOPS["fp64"] - 256 * 4 * 16 * 2 * 2.4e9 / 1e12) < 0.1
    assert abs(b.PEAK_TFLOPS["mixed"] - 157.3) < 0.1 and b.PEAK_TFLOPS["split"] == b.PEAK_TFLOPS["fp64"]
    assert b.FLOPS_PER_INTERACTION == {4: 60, 6: 97, 8: 144}


def test_counter_table_matches_sources_and_shapes():
    b = _bench_module()
    for prec in ("fp64", "mixed", "split"):
        t = b.MEASURED_COUNTERS[prec]
        h = b.kernel_sources_hash(t["launch"]["j_source"])
        assert t["valu_instr_per_pair"] > 0 and t["fp64_flops_per_pair"] > 0
        ex = b.executed_work(prec, t["launch"], 16384, 5e-4, 3e13)
        if t["sources_sha256"] == h:
            pairs = 16384 * 16383 / 2
            assert abs(ex["fp64_tflops"] - t["fp64_flops_per_pair"] * pairs / 5e-4 / 1e12) < 1e-9
        else:
            assert ex is None
        other = dict(t["launch"], j_source="lds")
        assert b.executed_work(prec, other, 16384, 5e-4, 3e13) is None


def test_oracle_used_only_in_the_cpu_baseline_leg():
    # the oracle is test infrastructure: bench.py may touch it only inside
    # its cpu_baseline leg
    import ast

    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    uses = []
    for fn in ast.walk(tree):
        if not isinstance(fn, ast.FunctionDef):
            continue
        for node in ast.walk(fn):
            mod = None
            if isinstance(node, ast.ImportFrom):
                mod = node.module
            elif isinstance(node, ast.Import):
                mod = node.names[0].name
            if mod and mod.split(".")[0] == "oracle":
                uses.append(fn.name)
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    assert not any((getattr(n, "module", None) or n.names[0].name).split(".")[0] == "oracle" for n in top)
    assert set(uses) == {"cpu_baseline"}, uses
