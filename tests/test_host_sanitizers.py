"""Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU needed): every translation unit of paper_2503_15259_amd/csrc/psca.hip
is compiled for the host only, with the sanitizers on the host pass and an
empty embedded device binary, linked into a shared library, and exercised by
tests/native/host_abi_check.c (argument checks of every entry point, context
creation on a device that does not exist, status strings), with leak
detection on and every UBSan report fatal."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCE = os.path.join(ROOT, "paper_2503_15259_amd", "csrc", "psca.hip")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "native", "host_abi_check.c")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
UNITS = [["-DPSCA_TU_MAIN"]] + [["-DPSCA_TU_BACK", f"-DPSCA_BACK_LO={lo}", f"-DPSCA_BACK_HI={hi}"]
                                 for lo, hi in ((5, 10), (11, 13), (14, 15), (16, 16))]
# the sanitizers go to the host pass only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    empty = tmp_path / "empty.bin"
    empty.write_bytes(b"")
    procs, objs = [], []
    for k, defs in enumerate(UNITS):
        obj = tmp_path / f"tu{k}.o"
        objs.append(str(obj))
        cmd = [HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-Xclang", "-fcuda-include-gpubinary",
               "-Xclang", str(empty), "-O1", "-g", "-fPIC", "-std=c++17", *SAN, "-I", INCLUDE, *defs,
               "-c", SOURCE, "-o", str(obj)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    lib = tmp_path / "libpsca_san.so"
    subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN, "-shared", "-fPIC", *objs, "-o", str(lib)],
                   check=True, capture_output=True, text=True)
    exe = tmp_path / "host_abi_check"
    subprocess.run([CLANG, "-fsanitize=address,undefined", "-g", "-I", INCLUDE, DRIVER, "-L", str(tmp_path),
                    "-lpsca_san", f"-Wl,-rpath,{tmp_path}", "-o", str(exe)], check=True, capture_output=True,
                   text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    report = res.stdout + res.stderr
    assert res.returncode == 0, report
    assert "host ABI checks passed" in report
    for marker in ("AddressSanitizer", "LeakSanitizer", "runtime error"):
        assert marker not in report, report
