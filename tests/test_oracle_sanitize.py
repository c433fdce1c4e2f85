"""The oracle under AddressSanitizer, UndefinedBehaviorSanitizer and leak detection: a g++
build of amg_oracle.cpp with the driver oracle/sanitize_main.cpp, which runs every entry
point on small ragged problems (setup, the three update modes and the rebuild policy, CG and
BiCGStab, exports, prescribed transfer operators, plain aggregation with SPAI0, a system of
2 x 2 blocks, the log-coefficient assembly and adjoint, argument errors).  Host code only;
the OpenMP pragmas are left out of this build (serial)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "ora_san")
    cmd = ["g++", *FLAGS, os.path.join(ORACLE, "amg_oracle.cpp"), os.path.join(ORACLE, "sanitize_main.cpp"),
           "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtimes not installed")
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-6000:])
    assert "all checks passed" in run.stdout
