"""Host-side checks of the benchmark (no GPU needed): more than one GPU is refused with a
one-line JSON message and exit status 2, before any device is touched; the HBM-traffic figure
the benchmark reports is the one its committed counter summary measured."""
import importlib.util
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_help_lists_the_studies():
    r = run("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--serve", "--fill", "--dilution", "--point-study"):
        assert flag in r.stdout


def test_traffic_figure_is_its_profiles_measurement():
    """Each entry of the benchmark's traffic table (HBM bytes per launch of the dominant stencil,
    reported only while the stencil's sources hash to the value it was measured on) equals the
    figure of the counter summary it names, and that summary gives its command."""
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert bench.TRAFFIC
    for key, tr in bench.TRAFFIC.items():
        with open(os.path.join(ROOT, tr["profile"])) as fh:
            text = fh.read()
        m = re.search(r"measured HBM bytes per launch ([0-9.]+e[+-]?[0-9]+)", text)
        assert m, (key, tr["profile"])
        assert abs(float(m.group(1)) - tr["bytes"]) <= 1e-3 * tr["bytes"], (key, m.group(1), tr["bytes"])
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
        assert re.fullmatch(r"[0-9a-f]{16}", tr["src"])
