"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the FP64
oracle (oracle/oracle7d.c, every entry point, tests/sanitize/oracle_driver.c)
and the library's planning (sd7_plan in csrc/api.hip on valid and invalid
frame sets, tests/sanitize/plan_driver.cpp).  The sanitizers instrument the
host side only; no GPU is used.  Any report aborts the program
(-fno-sanitize-recover), which fails the test."""
import os
import shlex
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = "-fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer"
# hipcc: each sanitizer flag goes to the host compilation only
HIP_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
           "-Xarch_host -fno-sanitize-recover=all -fno-omit-frame-pointer")


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_asan")
    cmd = (["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off"] + shlex.split(SAN)
           + ["-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_driver.c"),
              os.path.join(ROOT, "oracle", "oracle7d.c"), "-lm", "-o", exe])
    rc, out = _run(cmd)
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    assert "oracle driver:" in out


def test_planning_under_address_and_undefined_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc missing")
    exe = str(tmp_path / "plan_asan")
    cmd = ([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + shlex.split(HIP_SAN)
           + ["-I", os.path.join(ROOT, "include"), os.path.join(HERE, "plan_driver.cpp"),
              os.path.join(ROOT, "paper_2503_07946_amd", "csrc", "api.hip"), "-o", exe])
    rc, out = _run(cmd, timeout=600)
    assert rc == 0, out
    # the HIP runtime's own start-up allocations are not the planner's: no leak check
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    assert out.rstrip().endswith("0 failed"), out
