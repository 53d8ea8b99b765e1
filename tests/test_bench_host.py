"""Host logic of bench.py (CPU): the one-GPU rule of its command line and the
rocprofv3 summary that its roofline figures are read from."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert not any(line.startswith("{") for line in r.stdout.splitlines())


def _write_csv(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for row in rows:
            f.write(",".join(str(x) for x in row) + "\n")


def test_summary_of_kernel_stats_and_counters(tmp_path):
    b = _bench_module()
    trace = tmp_path / "trace"
    pmc = tmp_path / "pmc"
    trace.mkdir()
    pmc.mkdir()
    _write_csv(trace / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
               [["k_small", 4, 8000, 2000], ["k_big(int)", 2, 50000, 25000]])
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = [
        # two dispatches of k_big; the first reported in two parts (summed)
        [1, "k_big(int)", "FETCH_SIZE", 100.0], [1, "k_big(int)", "FETCH_SIZE", 50.0],
        [2, "k_big(int)", "FETCH_SIZE", 250.0],
        [1, "k_big(int)", "WRITE_SIZE", 30.0], [2, "k_big(int)", "WRITE_SIZE", 50.0],
        # the 1 GiB calibration copy: half of it counted by FETCH_SIZE, all by WRITE_SIZE
        [3, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0],
        [3, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0],
    ]
    _write_csv(pmc / "run_counter_collection.csv", hdr, rows)
    md = b.summarize_profiles([str(trace), str(pmc)])
    lines = md.splitlines()
    # kernels ordered by total time, averages in microseconds
    i_big = next(i for i, l in enumerate(lines) if l.startswith("| `k_big"))
    i_small = next(i for i, l in enumerate(lines) if l.startswith("| `k_small"))
    assert i_big < i_small
    assert "| 2 | 25.0 | 50.0 |" in lines[i_big]
    data = json.loads(md[md.index("```json") + 7:md.rindex("```")])
    assert data["sources_sha"] == b.sources_sha()
    assert data["fetch_scale"] == 2.0 and data["write_scale"] == 1.0
    kb = data["kernels"][b.kernel_key("k_big(int)")]
    assert kb["FETCH_SIZE_kib"] == 200.0  # (150 + 250) / 2 dispatches
    assert kb["WRITE_SIZE_kib"] == 40.0
