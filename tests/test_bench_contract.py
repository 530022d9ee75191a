"""The bench's host-side contract, without a GPU: it refuses more than one GPU
with a message (this library drives one), and the blend kernel's measured
HBM traffic is read from the committed counter summary only while the
kernel's sources are the ones the counters were taken on."""
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_summary_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    fields = dict(l.split(": ", 1) for l in open(bench.TRAFFIC_SUMMARY).read().splitlines() if ": " in l)
    sources = fields["kernel_sources"].split()
    assert float(fields["traffic_bytes_per_launch"]) > 0
    # a copy of the tree's kernel sources: same hash, same figure
    for s in sources:
        os.makedirs(tmp_path / os.path.dirname(s), exist_ok=True)
        shutil.copy(os.path.join(ROOT, s), tmp_path / s)
    os.makedirs(tmp_path / "profiles")
    shutil.copy(bench.TRAFFIC_SUMMARY, tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "profiles" / os.path.basename(bench.TRAFFIC_SUMMARY)))
    same = bench.measured_traffic()
    # one changed byte in a kernel source: no figure
    with open(tmp_path / sources[0], "a") as f:
        f.write("\n")
    changed = bench.measured_traffic()
    assert changed is None
    # the committed sources may be newer than the summary; then both are None
    assert same is None or same == float(fields["traffic_bytes_per_launch"])
