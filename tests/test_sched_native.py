"""The serving scheduler's device-free core (queue, footprint admission, batch
formation, worker threads, registration, shutdown) built with g++ on the CPU
under ThreadSanitizer and under AddressSanitizer + UndefinedBehaviorSanitizer,
driven by a stub executor (tests/native/sched_check.cpp): concurrent
submissions, registrations and releases, injected allocation failures, the
registered-system admission cases and shutdown with queued requests."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_check.cpp")
INC = os.path.join(ROOT, "paper_1912_01491_amd", "csrc")

SANITIZERS = {
    "thread": ["-fsanitize=thread"],
    "address_undefined": ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"],
}


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = {}
    d = tmp_path_factory.mktemp("sched")
    for name, flags in SANITIZERS.items():
        exe = str(d / ("sched_" + name))
        r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", *flags, "-I", INC, SRC, "-o", exe, "-lpthread"],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out[name] = exe
    return out


@pytest.mark.parametrize("san", sorted(SANITIZERS))
@pytest.mark.parametrize("scenario", ["stress", "registered", "late", "refuse", "shutdown", "oom", "group"])
def test_scheduler_under_sanitizer(binaries, san, scenario):
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    r = subprocess.run([binaries[san], scenario], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
