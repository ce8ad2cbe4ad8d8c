"""Host-side checks of bench.py: the one-GPU contract and the counter files
its roofline traffic is read from."""
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
    assert "one GPU" in r.stderr and r.stdout == ""


def _summary(tmp_path, digest, form=""):
    sfx = "_" + form if form else ""
    p = tmp_path / "counters.md"
    p.write_text("# counters\n\nValues:\n\n"
                 "    fetch_kib%s: 1000\n    write_kib%s: 500\n"
                 "    fetch_scale: 2.0\n    write_scale: 1.0\n"
                 "    source_sha256_16: %s\n" % (sfx, sfx, digest))
    return str(p)


def test_counter_traffic_scales_fetch_and_write(tmp_path):
    files = ["bench.py"]
    digest = bench.sources_hash(files)
    path = _summary(tmp_path, digest, "f16")
    assert bench.counter_traffic(path, files, "f16") == (1000 * 2.0 + 500 * 1.0) * 1024
    # a form the summary does not hold
    assert bench.counter_traffic(path, files, "plain") is None


def test_counter_traffic_is_null_once_sources_change(tmp_path):
    files = ["bench.py"]
    path = _summary(tmp_path, "0" * 16)
    assert bench.counter_traffic(path, files) is None
    assert bench.counter_traffic(str(tmp_path / "missing.md"), files) is None


@pytest.mark.parametrize("workload", sorted(bench.TRAFFIC_FILES))
def test_committed_counter_files_parse(workload):
    """Every committed fit counter summary holds the keys bench.py reads."""
    text = open(bench.TRAFFIC_FILES[workload]).read()
    keys = {ln.strip().split(":", 1)[0] for ln in text.splitlines()
            if ln.startswith("    ") and ":" in ln}
    assert {"fetch_scale", "write_scale", "source_sha256_16"} <= keys
    assert any(k.startswith("fetch_kib") for k in keys)
    assert any(k.startswith("write_kib") for k in keys)


def test_committed_valu_summary_parses():
    """The fit's VALU summary holds the issue rates bench.py reports, and they
    are plausible (saturated issue reads about one instruction per pass)."""
    text = open(bench.VALU_FILE).read()
    kv = {ln.strip().split(":", 1)[0]: ln.strip().split(":", 1)[1].strip()
          for ln in text.splitlines() if ln.startswith("    ") and ":" in ln}
    for form in ("plain", "f16"):
        assert 0.5 < float(kv["valu_issue_" + form]) < 2.0
    assert "source_sha256_16" in kv
