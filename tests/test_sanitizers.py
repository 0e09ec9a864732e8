"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds, in this process's container:
  * liblbm.so with its host code sanitized (paper_1510_07328_amd/build.py,
    build_sanitized: host compilation only, every sanitizer flag scoped to the
    host with -Xarch_host);
  * the oracle library (lbm_oracle.c, lbm_oracle_api.c) sanitized, compiled here
    by the ROCm clang so that both share one sanitizer runtime;
then runs the ABI tests and the oracle tests in a child process that preloads
clang's shared AddressSanitizer runtime and loads the sanitized libraries
($LBM_LIBRARY, $LBM_ORACLE_LIBRARY).  Any sanitizer report fails the run
(-fno-sanitize-recover=all, halt_on_error)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
ORACLE = os.path.join(ROOT, "oracle")
ORACLE_SANITIZED = os.path.join(ORACLE, "_build_sanitized", "liblbm_oracle.so")


def build_oracle_sanitized() -> str:
    os.makedirs(os.path.dirname(ORACLE_SANITIZED), exist_ok=True)
    srcs = [os.path.join(ORACLE, s) for s in ("lbm_oracle.c", "lbm_oracle_api.c")]
    cmd = [CLANG, "-O1", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
           "-o", ORACLE_SANITIZED, *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    return ORACLE_SANITIZED


def asan_runtime() -> str:
    path = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    assert os.path.exists(path), path
    return path


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not found")
def test_abi_and_oracle_tests_pass_under_asan_and_ubsan():
    from paper_1510_07328_amd import build as B

    lib = B.build_sanitized()
    orc = build_oracle_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": " ".join(p for p in (asan_runtime(), env.get("LD_PRELOAD", "")) if p),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "LBM_LIBRARY": lib,
        "LBM_ORACLE_LIBRARY": orc,
        "OMP_NUM_THREADS": "1",
    })
    tests = ["tests/test_abi.py", "tests/test_oracle_api.py", "tests/test_oracle_lbm.py",
             "tests/test_oracle_porous.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", *tests, "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        "-x"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "runtime error:" not in out
    assert r.returncode == 0
    assert " passed" in out
