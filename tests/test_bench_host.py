"""CPU checks of bench.py's host logic: the one-GPU contract and the guard that drops a
committed counter summary once the contraction kernel's sources no longer match it."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _summary(tmp_path, digest, extra):
    p = tmp_path / "summary.txt"
    p.write_text("# a comment=with an equals sign\n" + f"kernel_source_sha256_16={digest}\n" + extra)
    return str(p)


def test_profile_values_follow_the_kernel_sources(tmp_path, monkeypatch):
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    good = _summary(tmp_path, h.hexdigest()[:16], "hbm_bytes_per_launch=1234\n")
    monkeypatch.setattr(bench, "ROOT", "/")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [os.path.join(ROOT, f) for f in bench.KERNEL_SOURCES])
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", {"w": good})
    assert bench.profiled_traffic("w") == 1234
    assert bench.profiled_traffic("other") is None
    stale = _summary(tmp_path, "0" * 16, "hbm_bytes_per_launch=1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", {"w": stale})
    assert bench.profiled_traffic("w") is None


def test_committed_summaries_name_their_commands():
    for table in (bench.TRAFFIC_PROFILE, bench.MFMA_PROFILE):
        for path in table.values():
            text = open(os.path.join(ROOT, path)).read()
            assert "rocprofv3 --pmc" in text and "python3 bench.py" in text
            assert "kernel_source_sha256_16=" in text
