"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds, each loaded in a child process with its sanitizer runtime
preloaded and every report made fatal:
- the library with its host pass instrumented (argument checks, layouts,
  constant tables built with 512-bit integers, workspace queries, the knob
  table), running the host-only C-ABI tests of test_abi.py plus a sweep of
  the constant tables and workspace queries over every N, precision and
  moduli table;
- the C++ twin of the oracle, running its parity tests against the Python
  oracle.
No kernel is launched: device code is built as usual and never reached.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "hostsan")

SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
}

LIB_DRIVER = r"""
import ctypes, sys
sys.path.insert(0, sys.argv[1])
import pytest
import paper_2602_02549_amd as oz
oz.LIB_PATH = sys.argv[2]
L = oz.lib()
buf = (ctypes.c_double * 4096)()
p = (ctypes.c_int * 64)()
for prec in (64, 32, 16):
    for table in (0, 1, 2):
        for N in range(0, 52):
            L.ozaki2_debug_constants(prec, table, N, buf)
            L.ozaki2_moduli(table, N, p)
for prec in (64, 32):
    for s in [(0, 0, 0, 2), (1, 1, 1, 2), (300, 200, 500, 14), (64, 64, 262144, 14),
              (4096, 4096, 4096, 49), (5, 7, (1 << 19) - 1, 20), (5, 7, 1 << 19, 20), (-1, 3, 3, 3)]:
        oz.ozaki2_workspace_bytes(prec, *s)
        oz.ozaki2_complex_workspace_bytes(prec, *s)
        oz.ozaki2_certified_workspace_bytes(prec, *s)
    oz.ozaki2_batched_workspace_bytes(prec, [64, 64, 262144, 14] * 70 + [0, 5, 5, 5])
print("sweep done", flush=True)
sys.exit(pytest.main(["-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
                      sys.argv[1] + "/tests/test_abi.py"]))
"""

TWIN_DRIVER = r"""
import sys
sys.path.insert(0, sys.argv[1])
import pytest
import oracle.twin as tw
tw.LIB = sys.argv[2]
sys.exit(pytest.main(["-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
                      sys.argv[1] + "/tests/test_oracle_twin.py"]))
"""


def run_child(driver, lib, preload):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
    p = subprocess.run([sys.executable, "-c", driver, ROOT, lib], env=env, cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=900)
    out = p.stdout
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
    return out


def test_library_host_code_under_asan_ubsan():
    from paper_2602_02549_amd import build as b
    try:
        runtime = b.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = b.build_host_sanitized(OUT)
    out = run_child(LIB_DRIVER, lib, runtime)
    assert "sweep done" in out and " passed" in out


def test_oracle_twin_under_asan_ubsan():
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], stdout=subprocess.PIPE,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc ASan runtime not found")
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libos_ii_twin_san.so")
    src = os.path.join(ROOT, "oracle", "os_ii_twin.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                    "-shared", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", src, "-o",
                    lib], check=True)
    out = run_child(TWIN_DRIVER, lib, asan)
    assert " passed" in out
