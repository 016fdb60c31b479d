"""The benchmark's command-line contract, on the CPU: more than one GPU is
refused with a message, and the oracle-baseline child process (which never
touches the GPU) prints one JSON object with the fields the result line
carries."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_cpu_baseline_child_prints_its_result():
    r = subprocess.run([sys.executable, BENCH, "--cpu-baseline-child", "--n", "300", "--views", "1",
                        "--cpu-seconds", "1", "--cpu-procs", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["kind"] == "oracle" and d["unit"] == "Mpix/s" and d["cores"] == 2
    assert d["value"] > 0 and "pixels of view 0" in d["sample"]
