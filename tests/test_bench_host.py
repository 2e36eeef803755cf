"""Host-side checks of bench.py: the one-GPU guard of its command line and
the rule that the roofline's HBM traffic is reported only when the committed
counter summary was taken on the current kernel source.  No GPU."""
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _tree(tmp_path):
    """A copy of the kernel sources and the committed traffic summaries."""
    src = os.path.join(ROOT, "paper_2306_09559_amd", "csrc")
    dst = tmp_path / "paper_2306_09559_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, f), dst / f)
    (tmp_path / "profiles").mkdir()
    return dst


def _summary(tmp_path, prec, digest, traffic):
    (tmp_path / "profiles" / f"k_sweep_c2_{prec}_traffic.md").write_text(
        "# traffic\n\n"
        f"- kernel_source_hash: `{digest}`\n"
        f"- traffic_bytes_per_launch: {traffic}\n")


def test_traffic_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    digest = bench.kernel_source_hash()
    assert len(digest) == 16
    # no summary: no figure
    assert bench.measured_traffic("f64") is None
    _summary(tmp_path, "f64", digest, 466649303)
    assert bench.measured_traffic("f64") == 466649303
    # any change to a kernel source, a comment included, voids the figure
    f = csrc / bench.KERNEL_SOURCES[0]
    f.write_text(f.read_text() + "\n// edited\n")
    assert bench.kernel_source_hash() != digest
    assert bench.measured_traffic("f64") is None
    # a summary with no usable figure gives none either
    _summary(tmp_path, "f32", bench.kernel_source_hash(), "n/a")
    assert bench.measured_traffic("f32") is None


def test_committed_summaries_name_a_hash_and_a_figure():
    for prec in ("f64", "f32"):
        p = os.path.join(ROOT, "profiles", f"k_sweep_c2_{prec}_traffic.md")
        text = open(p).read()
        assert "kernel_source_hash:" in text and "traffic_bytes_per_launch:" in text
        assert "rocprofv3 --pmc" in text            # the command that made it
