"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle and the library's host code (geometry, context set-up,
argument validation, index sets, the server's queue) are rebuilt with
-fsanitize=address,undefined and the CPU test files that exercise them are
run against those builds in a child process with the ASan runtime
preloaded; any invalid access, overflow or undefined operation aborts the
child.  The device code objects are linked unchanged (they run only on a
GPU, and the host-only contexts of these tests never launch them)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_20252_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2512_20252_amd", "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _device_objects():
    objs = [os.path.join(BUILD, "kernels.o"), os.path.join(BUILD, "kernels_update2d_f64.o")]
    return objs if all(os.path.exists(o) for o in objs) else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None or _runtime("libubsan.so") is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    dev = _device_objects()
    if dev is None:
        pytest.skip("device objects not built (run __graft_entry__.build())")
    # the oracle, with its own flags plus the sanitizers
    orc = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-shared", "-fPIC"] + SAN +
                          ["-o", orc, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    # the library's host code, with its own flags plus the sanitizers
    host = ["-O1", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-D__HIP_PLATFORM_AMD__",
            "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs = []
    for src in ("geometry.cpp", "ibdvm.cpp", "server.cpp"):
        o = str(tmp_path / src.replace(".cpp", ".o"))
        subprocess.check_call(["g++"] + host + SAN + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    lib = str(tmp_path / "libibdvm_san.so")
    subprocess.check_call(["g++", "-shared", "-fPIC"] + SAN + ["-o", lib] + objs + dev +
                          ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    # reports go to files: pytest's capture would swallow a report written
    # to the stderr of a child that the sanitizer ends
    logs = tmp_path / "san"
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS=f"detect_leaks=0:log_path={logs}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={logs}", OMP_NUM_THREADS="2")
    files = ["tests/test_abi_cpu.py", "tests/test_oracle_pins_options.py", "tests/test_oracle_pins_refined.py"]
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_run.py"), orc, lib] + files,
                       env=env, capture_output=True, text=True, timeout=900)
    reports = "".join(open(f).read() for f in sorted(tmp_path.glob("san*")))
    assert r.returncode == 0 and not reports, (reports[:4000] or (r.stdout + r.stderr)[-4000:])
    assert " passed" in r.stdout, r.stdout[-2000:]
