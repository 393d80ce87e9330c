"""Host logic of the planner and the serving loop, on the CPU: libtcm's runtime and server
sources are compiled against a stand-in for the HIP runtime (tests/host/) with
AddressSanitizer and UndefinedBehaviorSanitizer, and driven with random request streams under
tight HBM budgets (admission, LRU eviction, deferral, fragments shared by several in-flight
launches, failure paths).  Every ticket must complete, every result must name the two
fragments of its request, and device memory must stay within the budget."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SRC = os.path.join(ROOT, "paper_0704_1672_amd", "csrc")


def _build(tmp_path, sanitize):
    exe = str(tmp_path / "server_stress")
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer",
           "-I", HOST, "-I", os.path.join(ROOT, "include"), "-I", SRC, "-o", exe,
           os.path.join(HOST, "server_stress.cpp"), os.path.join(HOST, "mock_hip.cpp"),
           os.path.join(SRC, "tcm_runtime.cpp"), os.path.join(SRC, "tcm_server.cpp"), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_server_stress_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "address,undefined")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, "12"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    # injected allocation and launch failures fail their own requests only, leak nothing,
    # and the server serves a clean batch afterwards
    faults = [l for l in r.stdout.splitlines() if l.startswith("faults:")]
    assert len(faults) == 1 and faults[0].endswith(" ok"), faults
    lines = [l for l in r.stdout.splitlines() if l.startswith("seed")]
    assert len(lines) == 12
    assert all(" bad 0 " in l and l.endswith("ok") for l in lines), lines


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_server_stress_tsan(tmp_path):
    """The serving loop (server thread, submitting and polling thread, launch slots) under
    ThreadSanitizer: no data race or lock misuse is reported."""
    exe = _build(tmp_path, "thread")
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, "4"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert len([l for l in r.stdout.splitlines() if l.startswith("seed")]) == 4


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_adaptive_plans_asan_ubsan(tmp_path):
    """Adaptive plans on the HIP stand-in under ASan/UBSan: every run equals the one-shot
    adaptive call, destroyed plans give their memory back, and creations failing under
    injected allocation failures leave the budget as it was."""
    exe = str(tmp_path / "adaptive_plan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I", HOST, "-I", os.path.join(ROOT, "include"), "-I", SRC, "-o", exe,
           os.path.join(HOST, "adaptive_plan.cpp"), os.path.join(HOST, "mock_hip.cpp"),
           os.path.join(SRC, "tcm_runtime.cpp"), os.path.join(SRC, "tcm_server.cpp"), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "adaptive plans ok" in r.stdout
