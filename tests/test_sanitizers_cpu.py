"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code.

1. The library's host-only code (paper_1303_4945_amd/csrc/host.cpp: geometries,
   handle registry, plan tables, argument validation) and the CPU oracle
   (oracle/sht_oracle.c) are compiled with g++/gcc -fsanitize=address,undefined
   into tests/sanitize_driver.cpp, which exercises them on small, degenerate and
   invalid cases; any sanitizer report fails the test.
2. The oracle's pin tests run again in a child interpreter with a sanitized
   build of the oracle library (the sanitizer runtimes preloaded).

Build recipe (the same commands by hand):
  gcc -std=c99 -O1 -g -fopenmp -fsanitize=address,undefined -fno-sanitize-recover=all -c oracle/sht_oracle.c
  g++ -std=c++17 -O1 -g -fopenmp -fsanitize=address,undefined -fno-sanitize-recover=all \\
      paper_1303_4945_amd/csrc/host.cpp tests/sanitize_driver.cpp sht_oracle.o -lm
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1", "-fopenmp"]


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _san_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    return env


def test_host_code_and_oracle_clean_under_asan_ubsan(tmp_path):
    _need("gcc")
    _need("g++")
    obj = tmp_path / "sht_oracle.o"
    subprocess.check_call(["gcc", "-std=c99", *SAN, "-c", os.path.join(ROOT, "oracle", "sht_oracle.c"),
                           "-o", str(obj)])
    exe = tmp_path / "driver"
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-Wall",
                           os.path.join(ROOT, "paper_1303_4945_amd", "csrc", "host.cpp"),
                           os.path.join(ROOT, "tests", "sanitize_driver.cpp"), str(obj), "-lm",
                           "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=_san_env(), timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "all checks passed" in r.stdout


def test_oracle_pins_under_asan_ubsan(tmp_path):
    _need("gcc")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-std=c99", *SAN, "-fPIC", "-shared",
                           os.path.join(ROOT, "oracle", "sht_oracle.c"), "-lm", "-o", str(lib)])
    rt = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
        if not os.path.isabs(p):
            pytest.skip(f"{name} not found")
        rt.append(p)
    env = _san_env()
    env["ASAN_OPTIONS"] = env["ASAN_OPTIONS"].replace("detect_leaks=1", "detect_leaks=0")
    env["LD_PRELOAD"] = ":".join(rt + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["SHT_ORACLE_SO"] = str(lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", "not slow"],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
