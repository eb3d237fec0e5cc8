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


def test_parity_recheck_accepts_the_oracle_and_rejects_a_change():
    """The bench's in-run re-check: a device state equal to the oracle's
    passes, one cell off by 1e-10 (relative) fails the FP64 bar, and an L1
    error above 1e-5 fails the mixed bar."""
    import numpy as np

    from oracle import oracle as O
    from paper_2607_20704_amd import inputs as I
    b = load_bench()
    w = I.sod_uniform()
    T = O.Tree(w.ijkl, w.bc)
    ref = T.permute_cells(w.u)
    dts = T.run(ref, w.gamma, w.cfl, 2)
    cases = {"sod_l5": (w, 2, ("steps", 1), {"fp64": (ref.copy(), dts.copy()), "mixed": (ref.copy(), dts.copy())})}
    base, par = b.cpu_baseline(cases, 0)
    assert par["ok"] and par["cases"]["sod_l5"]["fp64_worst_ratio"] == 0.0
    assert base["kind"] == "oracle" and base["cores"] >= 1 and base["serial"]["cores"] == 1
    assert base["value"] > 0 and base["serial"]["value"] > 0
    bad = ref.copy()
    bad[1000, 0] *= 1 + 1e-10
    cases["sod_l5"] = (w, 2, ("steps", 1), {"fp64": (bad, dts.copy())})
    _, par = b.cpu_baseline(cases, 0)
    assert not par["ok"] and not par["cases"]["sod_l5"]["fp64_ok"]
    off = ref.copy()
    off[:, 4] *= 1 + 1e-4
    cases["sod_l5"] = (w, 2, ("steps", 1), {"mixed": (off, dts.copy())})
    _, par = b.cpu_baseline(cases, 0)
    assert not par["ok"] and not par["cases"]["sod_l5"]["mixed_ok"]
    assert np.isclose(par["cases"]["sod_l5"]["mixed_l1"][4], 1e-4, rtol=1e-6)
