"""Host code under the sanitizers (CPU).

The library's host FP64 plan (plan.cpp: check points, image tables,
pseudo-inverse, sphere maps, input validation) is compiled with g++ and the
sanitizers together with a driver that builds plans for both geometries,
both near sets and both surface rules, feeds invalid parameters and inputs,
and checks the plans' structural invariants.  Device code is not involved
(GPU sanitizers are not available for it here)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_plan_under_asan_ubsan():
    tmp = tempfile.mkdtemp(prefix="hsma_san_")
    try:
        exe = os.path.join(tmp, "host_plan_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               os.path.join(ROOT, "tests", "native", "host_plan_check.cpp"),
               os.path.join(ROOT, "paper_2104_05260_amd", "csrc", "plan.cpp"), "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
        assert "host plan checks passed" in run.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_server_core_under_sanitizers(san):
    """The serving core (queue, admission, completion, cancellation,
    shutdown; paper_2104_05260_amd/csrc/server_core.h) driven on the CPU by a
    fake backend that completes work from its own thread: 8 submitting and
    waiting threads, launch failures, a full queue, shutdown with queued and
    running requests, waiters blocked during destruction."""
    tmp = tempfile.mkdtemp(prefix="hsma_core_")
    try:
        exe = os.path.join(tmp, "server_core_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}",
               "-fno-sanitize-recover=all", "-pthread",
               "-I", os.path.join(ROOT, "paper_2104_05260_amd", "csrc"),
               os.path.join(ROOT, "tests", "native", "server_core_check.cpp"), "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
        for _ in range(3):
            run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
            assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
            assert "server core checks passed" in run.stdout
            assert "WARNING" not in run.stderr
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_server_flow_under_sanitizers(san):
    """The request server's host code end to end (server.cpp compiled on the
    CPU against a stand-in for the HIP runtime, tests/native/fake_hip, and a
    stand-in plan, tests/native/fake_device.h): one slot and eight, all
    requests at once and spread arrivals, four submitting threads, declared
    and request-created plan classes whose arenas differ, device-resident
    replicas with system ids and ready events (slot affinity and step
    replays counted), shutdown with queued requests; every result checked
    against the stand-in plan's closed form."""
    tmp = tempfile.mkdtemp(prefix="hsma_flow_")
    try:
        csrc = os.path.join(tmp, "pkg", "csrc")
        inc = os.path.join(tmp, "include")
        os.makedirs(csrc)
        os.makedirs(inc)
        src = os.path.join(ROOT, "paper_2104_05260_amd", "csrc")
        for f in ("server.cpp", "server_core.h"):
            shutil.copy(os.path.join(src, f), csrc)
        shutil.copy(os.path.join(ROOT, "tests", "native", "fake_device.h"), os.path.join(csrc, "device.h"))
        for f in ("hsma.h", "hsma_server.h"):
            shutil.copy(os.path.join(ROOT, "include", f), inc)
        exe = os.path.join(tmp, "server_flow_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}",
               "-fno-sanitize-recover=all", "-pthread", "-I", os.path.join(ROOT, "tests", "native", "fake_hip"),
               os.path.join(csrc, "server.cpp"), os.path.join(ROOT, "tests", "native", "server_flow_check.cpp"),
               "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
        assert "server flow checks passed" in run.stdout
        assert "WARNING" not in run.stderr
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
