"""Host code under the address and undefined-behaviour sanitizers (CPU only, no GPU).

* The C ABI's argument checks (``paper_1605_01799_amd/csrc/checks.cpp``: descriptors, the
  32-bit column limit npts * K < 2^31 of hopf_eval / hopf_closest_point / hopf_eval_ragged, and
  the ragged-batch routing rules) are built with g++ and ``-fsanitize=address,undefined`` into a
  driver that calls them with valid and invalid arguments and never launches a kernel.
* The FP64 oracle (``oracle/hopf_oracle.c``) is built with gcc and the same sanitizers into a
  driver that runs every Hamiltonian / initial-data kind, unions and both distance routes on one
  and several threads.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1", "-pthread"]


def _run(cmd_build, exe):
    subprocess.run(cmd_build, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "PASSED" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_abi_host_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    out = _run(["g++", "-std=c++17", *SAN, "-o", exe, os.path.join(TESTS, "host_checks_main.cpp"),
                os.path.join(ROOT, "paper_1605_01799_amd", "csrc", "checks.cpp")], exe)
    assert "npts = 2^31, K = 1" in out and "ragged: sqrt(<p, D p>) refined" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    out = _run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-o", exe, os.path.join(TESTS, "oracle_sanitize_main.c"),
                os.path.join(ROOT, "oracle", "hopf_oracle.c"), "-lm", "-lpthread"], exe)
    assert out.count("ok eval") == 32  # 6 H x 3 J x 2 thread counts, less ||.||_A with the squared norms
