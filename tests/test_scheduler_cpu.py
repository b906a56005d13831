"""The serving scheduler's host policy (paper_1910_01070_amd/csrc/serve_sched.h:
first-fit device arena, first-in first-out admission under a byte budget and
a slot cap) against a reference model in a mock executor, compiled with g++
under AddressSanitizer and UndefinedBehaviorSanitizer (tests/native/sched_check.cpp)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_policy_against_reference_model(tmp_path):
    exe = str(tmp_path / "sched_check")
    env = {k: v for k, v in os.environ.items() if k != "LD_PRELOAD"}
    build = subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-I" + os.path.join(ROOT, "paper_1910_01070_amd", "csrc"),
         os.path.join(ROOT, "tests", "native", "sched_check.cpp"), "-o", exe],
        capture_output=True, text=True, env=env, timeout=300)
    assert build.returncode == 0, build.stdout + build.stderr
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "scheduler policy checks passed" in run.stdout
