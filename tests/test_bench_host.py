"""Host-side logic of bench.py: the traffic figure's staleness check, the byte
accounting and the one-GPU guard (no GPU needed)."""
import importlib.util
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bytes_per_particle_at_27_modes():
    b = load_bench()
    assert b.p2g_bytes_per_particle(27) == 340      # x, perm or mass, coefficients
    assert b.g2p_bytes_per_particle(27) == 348      # x read, coefficients and x written
    assert b.g2p2g_bytes_per_particle(27) == 352    # x, perm read; x, coefficients written


def make_tree(tmp_path):
    """A copy of the kernel sources and headers the digest covers, plus a profiles dir."""
    b = load_bench()
    for rel in list(b.KERNEL_SOURCES.values()) + list(b.KERNEL_HEADERS):
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    (tmp_path / "profiles").mkdir()
    b.ROOT = str(tmp_path)
    b.PROFILES = str(tmp_path / "profiles")
    return b


def write_traffic(b, kernel, sha, value=1.25e9):
    path = os.path.join(b.PROFILES, f"traffic_{kernel}_wl.txt")
    with open(path, "w") as f:
        f.write(f"# comment = ignored\nkernel = {kernel}\nsource_sha = {sha}\n"
                f"bytes_per_launch = {value}\n")


def test_traffic_is_read_while_the_sources_match(tmp_path):
    b = make_tree(tmp_path)
    write_traffic(b, "g2p2g", b.source_digest("g2p2g"))
    assert b.measured_traffic("g2p2g", "wl") == 1.25e9
    assert b.measured_traffic("g2p2g", "other_workload") is None


@pytest.mark.parametrize("changed", ["kernel", "header"])
def test_traffic_goes_stale_when_a_source_changes(tmp_path, changed):
    b = make_tree(tmp_path)
    write_traffic(b, "g2p2g", b.source_digest("g2p2g"))
    rel = b.KERNEL_SOURCES["g2p2g"] if changed == "kernel" else b.KERNEL_HEADERS[0]
    with open(tmp_path / rel, "a") as f:
        f.write("\n// edited\n")
    assert b.measured_traffic("g2p2g", "wl") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
