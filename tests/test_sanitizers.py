"""Host-side sanitizer runs (CPU only): the oracle built with AddressSanitizer
and UndefinedBehaviorSanitizer runs its whole pin suite (tests/test_oracle.py)
in a child interpreter, and the request server's policy simulation
(tests/sched_sim.cpp over ct_sched.h) runs built with both.  Any report
fails the run (halt on the first error)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "libct_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra", *SAN, "-o", lib,
                           os.path.join(ROOT, "oracle", "ct_oracle.c")])
    asan_rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, **ENV_SAN, CT_ORACLE_LIB=lib)
    # the uninstrumented interpreter loads the instrumented oracle: the ASan
    # runtime has to come first (anything already preloaded stays, after it)
    env["LD_PRELOAD"] = asan_rt + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_scheduler_simulation_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sched_sim_san")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", *SAN,
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2311_04406_amd", "csrc"),
                           "-o", exe, os.path.join(ROOT, "tests", "sched_sim.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=dict(os.environ, **ENV_SAN))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert r.stdout.count("ok sched") == 6 and r.stdout.count("ok arena") == 3
