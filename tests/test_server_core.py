"""The request server's scheduling core on the CPU, driven by a fake executor.

The core (queues, admission by device memory, completion, cancellation) is plain
C++; tests/server_core_driver.cpp links it with worker threads that sleep instead
of solving and a free-memory figure that changes without telling the core.  Built
with clang++ under ThreadSanitizer when the toolchain has it (g++ otherwise).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_10672_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "server_core_driver.cpp")

SCENARIOS = ["lost_wakeup", "lost_wakeup_without_recheck", "busy", "budget_serialises",
             "budget_overlap", "small_batches", "cancel", "wait_timeout", "stress"]


def _compiler():
    clang = "/opt/rocm/llvm/bin/clang++"
    if os.path.exists(clang):
        return [clang, "-fsanitize=thread"], True
    return [shutil.which("g++") or "g++"], False


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("server_core") / "driver")
    cc, tsan = _compiler()
    subprocess.check_call(cc + ["-std=c++17", "-O1", "-g", "-pthread", "-I", CSRC, DRIVER,
                                os.path.join(CSRC, "server_core.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    return r, tsan


@pytest.mark.parametrize("name", SCENARIOS)
def test_scenario(driver_output, name):
    r, _ = driver_output
    lines = [ln for ln in r.stdout.splitlines() if ln.split()[1:2] == [name]]
    assert lines, r.stdout + r.stderr
    assert lines[0].startswith("PASS"), lines[0]


def test_no_data_race(driver_output):
    r, tsan = driver_output
    assert r.returncode == 0, r.stdout + r.stderr
    if tsan:
        assert "ThreadSanitizer" not in r.stderr, r.stderr[:4000]
