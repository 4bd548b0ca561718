"""bench.py's host-side contract (no GPU): the one-GPU refusal, the modes it offers, and
that the recorded HBM-traffic figures name the sources they were measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_one_json_line():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_modes_are_offered():
    r = _run("--help")
    assert r.returncode == 0
    for m in ("solve", "solves", "apply", "serve", "config", "oracle"):
        assert m in r.stdout


def test_traffic_record_is_tied_to_source_hashes():
    sys.path.insert(0, ROOT)
    import bench
    mt = bench.MEASURED_TRAFFIC
    assert len(mt["sources_sha256"]) == 64
    for key in ("forward_f32", "forward_s3"):
        assert mt[key]["launches_per_apply"] > 0
    assert len(bench.sources_sha256()) == 64
