"""Host-side logic of bench.py, no GPU: the one-GPU contract and the rule that the
profiled HBM traffic is reported only for the kernel sources it was measured on."""

import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def _tree(tmp_path):
    """A copy of the kernel sources and the traffic profile under tmp_path."""
    csrc = tmp_path / "paper_1503_03295_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("sco_kernels.hip", "sco_internal.h"):
        shutil.copy(os.path.join(ROOT, "paper_1503_03295_amd", "csrc", name), csrc / name)
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "k_step_L2304_traffic.md"), tmp_path / "profiles")
    return csrc


def test_traffic_follows_the_kernel_source_hash(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_source_hash()
    profile = (tmp_path / "profiles" / "k_step_L2304_traffic.md").read_text()
    recorded = [line.split(": ", 1)[1].strip() for line in profile.splitlines()
                if line.startswith("source_sha256: ")]
    assert len(recorded) == 1
    if recorded[0] != h:  # the committed profile predates the sources: no figure
        assert bench.measured_traffic() is None
        return
    t = bench.measured_traffic()
    assert t is not None and t > 0
    # a comment does not change the kernel, so the figure stands
    kern = csrc / "sco_kernels.hip"
    kern.write_text(kern.read_text() + "\n// a note\n/* another\n   note */\n")
    assert bench.kernel_source_hash() == h
    assert bench.measured_traffic() == t
    # a code change does
    kern.write_text(kern.read_text() + "\nnamespace { constexpr int kUnused = 1; }\n")
    assert bench.kernel_source_hash() != h
    assert bench.measured_traffic() is None
