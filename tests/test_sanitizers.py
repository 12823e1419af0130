"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The oracle is rebuilt with ``-fsanitize=address,undefined`` (gcc, errors
  fatal) and its pins run against that build in a child process with the
  sanitizer runtime preloaded.
* The HIP library is rebuilt with the sanitizers on its host code only
  (each ``-fsanitize=`` after ``-Xarch_host``; the gfx950 device code is
  compiled as usual) and the ABI tests -- symbol table, descriptor layout,
  argument validation, all without a GPU -- run against it the same way.

A sanitizer report makes the child exit non-zero, which fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
}


def _child(tests, env_extra, timeout):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", *tests, "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    lib = str(tmp_path / "liblbo_san.so")
    here = os.path.dirname(oracle.__file__)
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-fPIC", "-shared", "-I", here, "-o", lib,
                    os.path.join(here, "lbo.c"), os.path.join(here, "lbo3.c"), "-lm"],
                   check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    out = _child(["tests/test_oracle_pins.py", "tests/test_oracle3_pins.py",
                  "tests/test_oracle_window.py"], {"LBO_LIB": lib, "LD_PRELOAD": asan}, 900)
    assert " passed" in out


def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_1411_7051_amd import build as hipbuild
    lib = str(tmp_path / "liblbk_san.so")
    srcs = [os.path.join(hipbuild.CSRC, s) for s in hipbuild.SOURCES]
    subprocess.run([hipbuild.hipcc(), *hipbuild.FLAGS, "-g",
                    "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all",
                    "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", hipbuild.INCLUDE, "-o", lib, *srcs, *hipbuild.libs()],
                   check=True, capture_output=True)
    rt = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "lib", "clang")
    found = [os.path.join(d, f) for d, _, fs in os.walk(rt) for f in fs
             if f == "libclang_rt.asan-x86_64.so"]
    if not found:
        pytest.skip("clang ASan runtime not found")
    out = _child(["tests/test_abi.py"], {"LBK_LIB": lib, "LD_PRELOAD": found[0]}, 600)
    assert " passed" in out
