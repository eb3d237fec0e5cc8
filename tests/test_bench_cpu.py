"""Host logic of the benchmark script (no GPU): the one-GPU contract and the
counter summary that is used only while the kernel source it was taken on is
unchanged."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_follows_the_kernel_digest(tmp_path, monkeypatch):
    b = load_bench()
    digest = b.kernel_source_digest()
    assert len(digest) == 16 and int(digest, 16) >= 0
    f = tmp_path / "traffic.md"
    f.write_text("kernel_source_digest: %s\ntraffic_bytes_per_launch_fp64: 1.5e9\n"
                 "traffic_bytes_per_launch_mixed: 2.5e9\n" % digest)
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.measured_traffic("fp64") == 1.5e9
    assert b.measured_traffic("mixed") == 2.5e9
    f.write_text("kernel_source_digest: %s\ntraffic_bytes_per_launch_fp64: 1.5e9\n" % ("0" * 16))
    assert b.measured_traffic("fp64") is None
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert b.measured_traffic("fp64") is None


def test_digest_ignores_comments(tmp_path, monkeypatch):
    """A comment or blank-line edit keeps the digest; a code edit changes it."""
    b = load_bench()
    src = os.path.join(ROOT, "paper_2607_20704_amd", "csrc")
    names = ("rg_brick.hip", "rg_brick.hpp", "rg_math.hpp", "rg_internal.hpp")
    csrc = tmp_path / "paper_2607_20704_amd" / "csrc"
    csrc.mkdir(parents=True)
    for n in names:
        (csrc / n).write_text(open(os.path.join(src, n)).read())
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    d0 = b.kernel_source_digest()
    assert d0 == load_bench().kernel_source_digest()
    p = csrc / "rg_brick.hpp"
    p.write_text(p.read_text() + "\n// a remark\n/* a block\n   remark */\n\n")
    assert b.kernel_source_digest() == d0
    p.write_text(p.read_text() + "static int unused_marker = 1;\n")
    assert b.kernel_source_digest() != d0
