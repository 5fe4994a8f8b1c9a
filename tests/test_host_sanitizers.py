"""Host code under the sanitizers (CPU only, no GPU).

* The serving core (``paper_2311_17174_amd/csrc/server_core.hpp``: arena,
  request queue, continuous batching, admission, scheduler thread) on a
  simulated device, built with AddressSanitizer + UndefinedBehaviorSanitizer
  and, separately, ThreadSanitizer (``tests/host/server_core_test.cpp``).
* The CPU oracle on small inputs in every orbit convention and integrator,
  built with AddressSanitizer + UndefinedBehaviorSanitizer
  (``tests/host/oracle_driver.c``).

Every sanitizer report aborts the program (``-fno-sanitize-recover``), so a
report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
CSRC = os.path.join(ROOT, "paper_2311_17174_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc/g++ with the sanitizer runtimes")


def build_and_run(tmp_path, compiler, flags, src, name, args=(), env=None):
    exe = str(tmp_path / name)
    subprocess.check_call([compiler, *flags, src, "-o", exe,
                           *(["-lm"] if src.endswith(".c") else [])])
    e = dict(os.environ)
    e.update(env or {})
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=600, env=e)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "ALL OK" in r.stdout
    return r.stdout


@pytest.mark.parametrize("seed", ["1", "2"])
def test_server_core_asan_ubsan(tmp_path, seed):
    out = build_and_run(tmp_path, "g++",
                        ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall",
                         "-Wextra", "-Werror", "-pthread", "-I", CSRC],
                        os.path.join(HOST, "server_core_test.cpp"), "sct_asan", [seed])
    assert "split arena ok" in out


@pytest.mark.parametrize("seed", ["1", "2"])
def test_server_core_tsan(tmp_path, seed):
    build_and_run(tmp_path, "g++",
                  ["-std=c++17", "-O1", "-g", "-fsanitize=thread", "-Wall", "-Werror",
                   "-pthread", "-I", CSRC],
                  os.path.join(HOST, "server_core_test.cpp"), "sct_tsan", [seed],
                  env={"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})


def test_oracle_asan_ubsan(tmp_path):
    build_and_run(tmp_path, "gcc",
                  ["-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall",
                   "-Wno-unknown-pragmas"],
                  os.path.join(HOST, "oracle_driver.c"), "oracle_asan",
                  env={"OMP_NUM_THREADS": "2"})
