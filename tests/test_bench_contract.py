"""CPU tests of bench.py's host logic: the --gpus guard and the rule that
ties the reported HBM traffic to the counted kernels and operator."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _profile(tmp_path, sources, digest, traffic=123.0, algorithmic=456.0):
    p = tmp_path / "traffic.txt"
    p.write_text(
        "a summary line\n"
        f"kernel_source_sha256: {digest}\n"
        f"kernel_sources: {' '.join(sources)}\n"
        f"gather_G_traffic_bytes: {traffic}\n"
        f"gather_G_algorithmic_bytes: {algorithmic}\n")
    return str(p)


def test_traffic_reported_only_for_the_counted_kernels_and_operator(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, ["kernel.hip"], digest))
    assert bench.counted_traffic("gather_G_traffic_bytes", 456.0) == 123.0
    assert bench.counted_traffic("gather_G_traffic_bytes") == 123.0
    # another operator (algorithmic bytes differ): no traffic
    assert bench.counted_traffic("gather_G_traffic_bytes", 457.0) is None
    # a key without an entry: no traffic
    assert bench.counted_traffic("project_G_traffic_bytes", 1.0) is None
    # the kernel changed since the counters were taken: no traffic
    src.write_text("kernel source, edited\n")
    assert bench.counted_traffic("gather_G_traffic_bytes", 456.0) is None


def test_committed_traffic_profile_parses():
    """The committed summary names existing sources and carries the fields
    the bench reads (whether it matches the current tree is not asserted)."""
    fields = dict(l.split(": ", 1) for l in open(bench.TRAFFIC_PROFILE).read().splitlines() if ": " in l)
    for f in fields["kernel_sources"].split():
        assert os.path.exists(os.path.join(ROOT, f)), f
    assert float(fields["gather_G_traffic_bytes"]) > float(fields["gather_G_algorithmic_bytes"]) > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
