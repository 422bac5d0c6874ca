"""Host-side checks of the benchmark's bookkeeping (no GPU): every committed counter summary the
benchmark reads carries a machine line it can parse, naming the kernel class it is filed under,
and a stale source hash turns the figure off rather than reporting it."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

LINE = re.compile(r"^traffic_bytes_per_launch=(\d+)(?: traffic_per_algorithmic=([0-9.]+))? kernel=(\S+) "
                  r"sources_sha256=([0-9a-f]{64})$", re.M)


@pytest.mark.parametrize("kernel", sorted(bench.TRAFFIC))
def test_traffic_summary_has_a_machine_line(kernel):
    summary, sources = bench.TRAFFIC[kernel]
    text = open(os.path.join(ROOT, "profiles", summary)).read()
    m = LINE.search(text)
    assert m and m.group(3) == kernel
    assert int(m.group(1)) > 0
    if m.group(2):
        assert 0.5 < float(m.group(2)) < 2.0
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    for f in sources:
        assert os.path.exists(os.path.join(ROOT, f))


def test_stale_hash_gives_no_traffic(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    (prof / "s.md").write_text("traffic_bytes_per_launch=100 traffic_per_algorithmic=0.5 kernel=dots2 "
                               "sources_sha256=" + "0" * 64 + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC", {"dots2": ("s.md", ["k.hip"])})
    assert bench.measured_traffic("dots2", 1000.0) is None
    import hashlib
    h = hashlib.sha256(b"kernel source\n").hexdigest()
    (prof / "s.md").write_text(f"traffic_bytes_per_launch=100 traffic_per_algorithmic=0.5 kernel=dots2 sources_sha256={h}\n")
    assert bench.measured_traffic("dots2", 1000.0) == 500.0
    (prof / "s.md").write_text(f"traffic_bytes_per_launch=100 kernel=dots2 sources_sha256={h}\n")
    assert bench.measured_traffic("dots2", 1000.0) == 100.0
    assert bench.measured_traffic("spmv_arnoldi", 1000.0) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
