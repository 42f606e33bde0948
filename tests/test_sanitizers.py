"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the FP64 oracle (driven by tests/model/oracle_check.c over small lattices of
every kind it handles), the run-time radix schedule planner
(tests/model/sched_check.cpp) and the persistent launch's queue protocol
(tests/model/queue_model.cpp).  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "tests", "model")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=66",
           UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def build_and_run(tmp_path, name, cmd, args=(), timeout=300):
    exe = str(tmp_path / name)
    subprocess.check_call(cmd + ["-o", exe])
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=timeout,
                       env=ENV)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out and "runtime error" not in out, out
    return r.returncode, out


def test_oracle_asan_ubsan(tmp_path):
    rc, out = build_and_run(tmp_path, "oracle_check",
                            ["gcc", "-std=gnu11", *SAN, "-Wno-unknown-pragmas",
                             os.path.join(ROOT, "oracle", "lf2_oracle.c"),
                             os.path.join(MODEL, "oracle_check.c"), "-lm"])
    print(out.strip())
    assert rc == 0 and "0 failures" in out, out


def test_radix_schedules_asan_ubsan(tmp_path):
    rc, out = build_and_run(tmp_path, "sched_check",
                            ["g++", "-std=c++17", *SAN, os.path.join(MODEL, "sched_check.cpp")])
    assert rc == 0 and out.startswith("ok"), out


def test_queue_protocol_asan_ubsan(tmp_path):
    rc, out = build_and_run(tmp_path, "queue_model",
                            ["g++", "-std=c++20", *SAN, "-pthread",
                             os.path.join(MODEL, "queue_model.cpp")],
                            args=("ticket", 200, 17, 2, 4, 48, 8))
    print(out.strip().splitlines()[-1])
    assert rc == 0 and "errors=0" in out and "reset=1" in out, out
