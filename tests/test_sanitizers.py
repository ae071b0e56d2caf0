"""CPU sanitizer runs (no GPU).

* The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
  (float-to-int overflow included, every report fatal) runs the oracle's pin
  tests (tests/test_oracle_pins.py, tests/test_box_pins.py) in a child
  process with the sanitizer runtimes preloaded.
* The adjoint's LDS index arithmetic (tests/native/adj_index_replay.cpp: the
  kernels' own geometry functions from csrc/xrt_geom.h, compiled for the
  host) is replayed for random and edge-placed lines on several grids, under
  the same sanitizers, and every accumulator word must lie inside its row.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g"]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_adjoint_index_replay(tmp_path):
    exe = str(tmp_path / "adj_index_replay")
    src = os.path.join(ROOT, "tests", "native", "adj_index_replay.cpp")
    inc = os.path.join(ROOT, "paper_2503_20907_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", "-O1"] + SAN + ["-I", inc, "-o", exe, src])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "failures 0" in r.stdout
    assert "runtime error" not in r.stderr


def test_oracle_pins_under_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    import oracle
    lib = oracle.build(force=True, out=str(tmp_path / "liborc_san.so"), sanitize=True)
    env = dict(os.environ)
    env.update({"XRT_ORACLE_LIB": lib, "LD_PRELOAD": asan + ":" + ubsan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "OMP_NUM_THREADS": "4"})
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_box_pins.py")]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
