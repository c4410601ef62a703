"""The serving scheduler under sanitizers, on the CPU.

The scheduling core and the threaded loop the device server runs
(paper_2012_15797_amd/csrc/sched_core.hpp), the callback scheduler ABI
(sched.cpp) and the error state (gfc_error.cpp) contain no HIP code.  They
are built with tests/native/sched_check.cpp, which drives the policy through
gfc_sched_* on a simulated clock and the loop from several threads against a
simulated device, once with AddressSanitizer + UndefinedBehaviorSanitizer and
once with ThreadSanitizer; both runs must be clean.

The compiler is the ROCm LLVM clang++: GCC 11's ThreadSanitizer does not
intercept pthread_cond_clockwait, which libstdc++'s timed condition-variable
waits call, so it reports lock-protected accesses as races.  A control run
with the loop's poll() stripped of its lock must be reported."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_15797_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
SCHED_MAIN = os.path.join(ROOT, "tests", "native", "sched_check.cpp")
SOURCES = [os.path.join(CSRC, "sched.cpp"), os.path.join(CSRC, "gfc_error.cpp")]


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    pytest.skip("no clang++ with sanitizer runtimes")


def _build_and_run(tmp_path, san, csrc=CSRC):
    exe = tmp_path / f"sched_check_{san.replace(',', '_')}"
    cmd = [_clang(), "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-I", INCLUDE, "-I", csrc, SCHED_MAIN,
           *[os.path.join(csrc, os.path.basename(s)) for s in SOURCES], "-o", str(exe), "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=0")
    return subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_scheduler_is_clean_under_sanitizers(tmp_path, san):
    r = _build_and_run(tmp_path, san)
    assert r.returncode == 0 and "sched_check ok" in r.stdout, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "runtime error" not in r.stderr, r.stderr


def test_thread_sanitizer_sees_a_planted_race(tmp_path):
    """Control: the same check program against a copy of the core whose poll()
    reads the request table without the loop's lock."""
    src = tmp_path / "csrc"
    src.mkdir()
    for f in ("sched_core.hpp", "gfc_error.hpp", "sched.cpp", "gfc_error.cpp"):
        shutil.copy(os.path.join(CSRC, f), src / f)
    core = (src / "sched_core.hpp").read_text()
    locked = ("  gfc_status poll(uint64_t ticket, int* done, const float** out_dev, gfc_status* status_out) {\n"
              "    std::lock_guard<std::mutex> lock(mu_);\n")
    assert locked in core
    (src / "sched_core.hpp").write_text(core.replace(locked, locked.split("\n")[0] + "\n"))
    r = _build_and_run(tmp_path, "thread", csrc=str(src))
    assert "WARNING: ThreadSanitizer: data race" in r.stderr
