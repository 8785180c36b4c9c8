"""The request server's scheduling core and slot feeder on the CPU, with fakes.

The core (queues, admission by device memory, completion, cancellation) and the slot
feeder (continuous refill of the small-instance kernel) are plain C++.
tests/server_core_driver.cpp links the core with worker threads that sleep instead of
solving and a free-memory figure that changes without telling the core;
tests/slot_driver.cpp links the feeder with a fake device whose launches run the
device side of the slot protocol in threads.  Built with clang++ under
ThreadSanitizer when the toolchain has it (g++ otherwise).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_10672_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "server_core_driver.cpp")
SLOT_DRIVER = os.path.join(ROOT, "tests", "slot_driver.cpp")

SCENARIOS = ["lost_wakeup", "lost_wakeup_without_recheck", "busy", "budget_serialises",
             "budget_overlap", "small_batches", "cancel", "wait_timeout", "stress"]
SLOT_SCENARIOS = ["slot_refill", "slot_mid_launch", "slot_idle_relaunch",
                  "slot_launch_ends_on_its_own", "slot_launch_fails", "slot_shutdown",
                  "slot_stress"]


def _compiler():
    clang = "/opt/rocm/llvm/bin/clang++"
    if os.path.exists(clang):
        return [clang, "-fsanitize=thread"], True
    return [shutil.which("g++") or "g++"], False


def _build_and_run(tmp_path_factory, name, sources):
    exe = str(tmp_path_factory.mktemp(name) / "driver")
    cc, tsan = _compiler()
    subprocess.check_call(cc + ["-std=c++17", "-O1", "-g", "-pthread", "-I", CSRC] + sources +
                          ["-o", exe])
    return subprocess.run([exe], capture_output=True, text=True, timeout=120), tsan


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    return _build_and_run(tmp_path_factory, "server_core",
                          [DRIVER, os.path.join(CSRC, "server_core.cpp")])


@pytest.fixture(scope="module")
def slot_output(tmp_path_factory):
    return _build_and_run(tmp_path_factory, "slots",
                          [SLOT_DRIVER, os.path.join(CSRC, "server_core.cpp"),
                           os.path.join(CSRC, "slots.cpp")])


def _check(out, name):
    r, _ = out
    lines = [ln for ln in r.stdout.splitlines() if ln.split()[1:2] == [name]]
    assert lines, r.stdout + r.stderr
    assert lines[0].startswith("PASS"), lines[0]


@pytest.mark.parametrize("name", SCENARIOS)
def test_scenario(driver_output, name):
    _check(driver_output, name)


@pytest.mark.parametrize("name", SLOT_SCENARIOS)
def test_slot_scenario(slot_output, name):
    _check(slot_output, name)


@pytest.mark.parametrize("which", ["core", "slots"])
def test_no_data_race(driver_output, slot_output, which):
    r, tsan = driver_output if which == "core" else slot_output
    assert r.returncode == 0, r.stdout + r.stderr
    if tsan:
        assert "ThreadSanitizer" not in r.stderr, r.stderr[:4000]
