"""Host-side checks of bench.py: the one-GPU guard and the rule that the
profiled traffic and VALU figures are reported only for the kernel sources
they were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("matching", [True, False])
def test_traffic_is_tied_to_the_kernel_sources(tmp_path, monkeypatch, matching):
    sha = bench.kernel_sources_sha256()
    if not matching:
        sha = ("0" if sha[0] != "0" else "1") + sha[1:]
    p = tmp_path / "traffic.md"
    p.write_text("summary\n\nsweep_traffic_bytes=123456789 kernel_sources_sha256=%s\n" % sha)
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(p))
    assert bench.profiled_traffic() == (123456789 if matching else None)


def test_missing_traffic_profile_reads_as_unmeasured(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "absent.md"))
    assert bench.profiled_traffic() is None


@pytest.mark.parametrize("matching", [True, False])
def test_valu_busy_is_tied_to_the_kernel_sources(tmp_path, monkeypatch, matching):
    sha = bench.kernel_sources_sha256()
    if not matching:
        sha = ("0" if sha[0] != "0" else "1") + sha[1:]
    p = tmp_path / "counters.md"
    p.write_text("table\n\nsweep_valu_busy_pct=45.0 kernel_sources_sha256=%s\n" % sha)
    monkeypatch.setattr(bench, "COUNTERS_PROFILE", str(p))
    assert bench.profiled_valu_busy() == (45.0 if matching else None)


def test_kernel_hash_covers_every_sweep_source():
    csrc = os.path.join(ROOT, "paper_2606_04292_amd", "csrc")
    for name in bench.SWEEP_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name
    # every package header the FP64 kernel file includes, directly or not,
    # is hashed
    seen, todo = set(), ["kernels_fp64.hip"]
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        seen.add(name)
        with open(os.path.join(csrc, name)) as f:
            todo += [l.split('"')[1] for l in f if l.startswith('#include "')]
    assert seen <= set(bench.SWEEP_SOURCES), seen - set(bench.SWEEP_SOURCES)
