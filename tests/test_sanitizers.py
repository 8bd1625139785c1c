"""The oracle and the library's host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/sanitize/oracle_driver.c runs the oracle through every command and
accessor (two fluids with Shan-Chen forces, hybrid solids, momentum
openings, a D2Q9 solute with openings of every style on every wall,
reaction, growth and intersolute; one fluid with the psi forms and a D2Q4
solute).  tests/sanitize/abi_driver.c drives the host side of the C ABI
without a GPU (commands, order rules, argument checks, workspace layouts of
every storage format, refused binds and batches).  The runtime's host code
(lb2d_api.cpp) is built with the sanitizers; the launchers it links come
from the library's own build.  Both must exit cleanly with no sanitizer
report, leaks included."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert r.stdout.strip().endswith("ok")
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "LeakSanitizer" not in r.stderr


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fopenmp", *SAN, os.path.join(ROOT, "oracle", "lb2d_oracle.c"),
                           os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    _run(exe)


def test_host_runtime_under_sanitizers(tmp_path):
    from paper_1202_0442_amd import build as libbuild
    objs = [o for o in glob.glob(os.path.join(libbuild.HERE, "_build", "*.o")) if "lb2d_api" not in o]
    if len(objs) < len(libbuild.SOURCES) - 1:
        libbuild.build()
        objs = [o for o in glob.glob(os.path.join(libbuild.HERE, "_build", "*.o")) if "lb2d_api" not in o]
    api = str(tmp_path / "api_san.o")
    # device code as in the library; host code with the sanitizers
    host_san = [f for flag in SAN for f in ("-Xarch_host", flag)]
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", *host_san,
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", os.path.join(ROOT, "include"), "-I", libbuild.CSRC, "-x", "hip", "-c",
                           os.path.join(libbuild.CSRC, "lb2d_api.cpp"), "-o", api])
    clang = "/opt/rocm/llvm/bin/clang"
    drv = str(tmp_path / "abi_driver.o")
    subprocess.check_call([clang, *SAN, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "abi_driver.c"),
                           "-o", drv])
    exe = str(tmp_path / "abi_driver")
    subprocess.check_call([clang + "++", *SAN, drv, api, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                           "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    _run(exe)
