"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle (oracle/oracle.c) with a driver (oracle/sanitize_check.c) that runs
  every entry point on a ragged batch whose arrays are allocated at their exact sizes.
* The C ABI's host validation: the library's API translation unit rebuilt with the
  sanitizers on its host side only (device code is untouched), linked with the other
  objects, and driven by tests/abi_sanitize_main.cpp with invalid arguments.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"ASAN_OPTIONS": "abort_on_error=0:halt_on_error=1:exitcode=99",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=98",
           "OMP_NUM_THREADS": "2"}


def _run(cmd, env_extra=None, cwd=None, timeout=300):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=cwd, timeout=timeout)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    r = _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              os.path.join(ROOT, "oracle", "sanitize_check.c"), os.path.join(ROOT, "oracle", "oracle.c"),
              "-lm", "-o", exe])
    assert r.returncode == 0, r.stderr
    r = _run([exe], SAN_ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_abi_validation_under_address_and_ub_sanitizers(tmp_path):
    from paper_1604_06236_amd import build as B
    B.build(force=False)                      # the other objects, unsanitized
    obj = str(tmp_path / "bt_api_san.o")
    flags = [f for f in B.CFLAGS]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    r = _run([HIPCC] + flags + san + ["-c", os.path.join(B.CSRC, "bt_api.hip"), "-o", obj])
    assert r.returncode == 0, r.stderr
    others = sorted(os.path.join(B.BUILD, f) for f in os.listdir(B.BUILD)
                    if f.endswith(".o") and f != "bt_api.o")
    lib = str(tmp_path / "libblocktransform.so")
    r = _run([HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
              "-Xarch_host", "-fsanitize=undefined", "-o", lib, obj] + others)
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "abi_san")
    r = _run([HIPCC, "-std=c++17", "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", f"-I{os.path.join(ROOT, 'include')}",
              os.path.join(ROOT, "tests", "abi_sanitize_main.cpp"), "-o", exe, f"-L{tmp_path}",
              "-lblocktransform", f"-Wl,-rpath,{tmp_path}"])
    assert r.returncode == 0, r.stderr
    r = _run([exe], dict(SAN_ENV, ASAN_OPTIONS=SAN_ENV["ASAN_OPTIONS"] + ":detect_leaks=0"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
