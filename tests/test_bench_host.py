"""Host-side logic of bench.py: the one-GPU guard, the kernel source hash and
the reading of the committed HBM-traffic summary (no GPU needed)."""
import os
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
    assert "one GPU" in r.stderr


def test_kernel_source_hash_ignores_comments_and_whitespace(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("// a comment\nint f(int x)\n{\n    /* block\n comment */ return x + 1;  // trailing\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash(str(a)) == bench.kernel_source_hash(str(b))
    assert bench.kernel_source_hash(str(a)) != bench.kernel_source_hash(str(c))
    assert len(bench.kernel_source_hash(str(a))) == 16


def _fake_tree(tmp_path, code):
    src = tmp_path / "paper_2503_20907_amd" / "csrc"
    src.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        (src / name).write_text(code + "// " + name + "\n")
    (tmp_path / "profiles").mkdir()
    return [str(src / name) for name in bench.KERNEL_SOURCES]


def test_measured_traffic_reads_matching_lines_only(tmp_path, monkeypatch):
    srcs = _fake_tree(tmp_path, "int k;\n")
    sha = bench.kernel_source_hash(srcs)
    (tmp_path / "profiles" / "hbm_traffic_2048_cubic_fan_random.md").write_text(
        f"    traffic call=adjoint kernel=k_adjoint<3,1> count=1 sha={sha} read_bytes=100 write_bytes=20\n"
        f"    traffic call=adjoint kernel=k_adjoint<3,2> count=1 sha={sha} read_bytes=300 write_bytes=40\n"
        f"    traffic call=adjoint kernel=k_adj_reduce count=2 sha={sha} read_bytes=5 write_bytes=1\n"
        f"    traffic call=forward kernel=k_forward<3> count=1 sha={sha} read_bytes=7 write_bytes=1\n"
        f"    traffic call=adjoint kernel=k_adjoint<3,1> count=1 sha=0000000000000000 read_bytes=999 write_bytes=999\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("adjoint") == 472
    assert bench.measured_traffic("forward") == 8
    assert bench.measured_traffic("layout") is None
    # a code change (not a comment) invalidates the figures
    for p in srcs:
        with open(p, "a") as f:
            f.write("int j;\n")
    assert bench.measured_traffic("adjoint") is None


def test_flops_per_nonzero_counts_one_polynomial_and_one_fma():
    # degree 2n+1 Horner (2n+1 FMAs) plus the accumulation, 2 flops each
    assert [bench.flops_per_nonzero(n) for n in range(4)] == [4, 8, 12, 16]
