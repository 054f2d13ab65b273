"""Host logic of the benchmark (no GPU): the one-GPU contract, the device
code hash that ties the committed profiles to the kernels they were taken
on, the readers of those profiles, and the kernel-trace summary."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2 refused" in r.stderr
    assert r.stdout == ""


def _copy_sources(tmp_path):
    csrc = tmp_path / "paper_1802_09488_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_1802_09488_amd", "csrc", f), csrc / f)
    return csrc


def test_kernel_hash_covers_device_code_only(tmp_path, monkeypatch):
    """The hash changes with the kernels and their headers, not with the
    launches and the C ABI after probe.hip's host-side marker."""
    h0 = bench.kernel_source_hash()
    csrc = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    probe = csrc / "probe.hip"
    src = probe.read_bytes()
    k = src.find(bench.HOST_SIDE_MARKER)
    assert k > 0
    probe.write_bytes(src + b"\n// host-side edit\n")
    assert bench.kernel_source_hash() == h0
    probe.write_bytes(src[:k] + b"// device-side edit\n" + src[k:])
    assert bench.kernel_source_hash() != h0
    probe.write_bytes(src)
    (csrc / "geom.hpp").write_bytes((csrc / "geom.hpp").read_bytes() + b"\n")
    assert bench.kernel_source_hash() != h0


def test_profile_readers_follow_the_hash(tmp_path, monkeypatch):
    """Traffic and VALU figures are read from the counter summaries only
    when those were taken on the current device code."""
    h = bench.kernel_source_hash()
    traffic = tmp_path / "traffic.md"
    counters = tmp_path / "counters.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(counters))
    assert bench.measured_traffic() is None and bench.measured_valu() is None
    traffic.write_text("kernel sources sha256/16: `%s`\n\n"
                       "| probe_kernel exact | 2.705e+09 |\n| probe_kernel approx | 2.719e+09 |\n" % h)
    counters.write_text("kernel sources sha256/16: `%s`\n\n"
                        "| probe_kernel<3, 2, 0, 2, false, false> | 1048576 | 143.8 | 70.1 |\n"
                        "| probe_kernel<0, 2, 0, 2, false, false> | 1048576 | 139.5 | 66.0 |\n" % h)
    assert bench.measured_traffic() == {"exact": 2.705e9, "approx": 2.719e9}
    assert bench.measured_valu() == {"exact": 143.8, "approx": 139.5}
    stale = "0" * 16 if h != "0" * 16 else "1" * 16
    traffic.write_text(traffic.read_text().replace(h, stale))
    counters.write_text(counters.read_text().replace(h, stale))
    assert bench.measured_traffic() is None and bench.measured_valu() is None


def test_committed_profiles_name_a_hash_and_a_command():
    """Every committed summary says which device code it was taken on and
    the command that made it, which runs committed files only."""
    prof = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(prof) if f.endswith(".md"))
    assert names
    for f in names:
        txt = open(os.path.join(prof, f)).read()
        assert "kernel sources sha256/16: `" in txt, f
        assert "rocprofv3 " in txt and "bench.py" in txt, f
        assert "_work/" not in txt, f


def test_trace_summary(tmp_path, capsys):
    """Calls, average, minimum, maximum and total per (kernel, grid, block)."""
    d = tmp_path / "trace" / "host"
    d.mkdir(parents=True)
    rows = [("void act::probe_kernel<3, 2, 0, 2, false, false>(act::ProbeParams)", 1048576, 1024,
             1000, 1000 + 550_000),
            ("void act::probe_kernel<3, 2, 0, 2, false, false>(act::ProbeParams)", 1048576, 1024,
             5000_000, 5000_000 + 570_000),
            ("void act::resolve_list_kernel<0, false>(act::ProbeParams, unsigned int)", 1048576, 256,
             2000_000, 2000_000 + 37_000)]
    with open(d / "run_kernel_trace.csv", "w") as fh:
        fh.write("Kernel_Name,Grid_Size_X,Workgroup_Size_X,Start_Timestamp,End_Timestamp\n")
        for r in rows:
            fh.write('"%s",%d,%d,%d,%d\n' % r)
    bench.summarize_trace(str(tmp_path / "trace"))
    out = capsys.readouterr().out.splitlines()
    assert out[0].startswith("| kernel | grid (threads) | block | calls |")
    assert out[2] == "| probe_kernel<3, 2, 0, 2, false, false> | 1048576 | 1024 | 2 | 560.0 | 550.0 | 570.0 | 1.12 |"
    assert out[3] == "| resolve_list_kernel<0, false> | 1048576 | 256 | 1 | 37.0 | 37.0 | 37.0 | 0.04 |"
    with pytest.raises(SystemExit):
        bench.summarize_trace(str(tmp_path / "nothing"))
