"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/psca.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2503_15259_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "psca.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psca_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(N.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = N.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_version_and_strerror():
    lib = N.load()
    assert lib.psca_version() >= 100
    for code in (0, -1, -2, -3, -4, -5, 12345):
        assert isinstance(N.strerror(code), str) and N.strerror(code)
    assert "positive definite" in N.strerror(N.PSCA_ENOTPD)


def test_null_arguments_are_rejected_without_a_device():
    lib = N.load()
    prm = N.PscaParams()
    assert lib.psca_create(None, 0) == N.PSCA_EINVAL
    assert lib.psca_destroy(None) == N.PSCA_OK
    assert lib.psca_sample_cov(None, None, 4, 4, None, None) == N.PSCA_EINVAL
    assert lib.psca_sample_cov_batch(None, 2, None, 16, 4, 4, None, 16, None) == N.PSCA_EINVAL
    assert lib.psca_detect(None, None, None, 4, 4, ctypes.byref(prm), None, None, None) == N.PSCA_EINVAL
    assert lib.psca_detect_y(None, None, None, 4, 4, ctypes.byref(prm), None, None, None) == N.PSCA_EINVAL
    assert lib.psca_iterate(None, None, None, 4, 4, ctypes.byref(prm), ctypes.c_float(0.5), None, None,
                            None, None, None, None, None) == N.PSCA_EINVAL
    assert lib.psca_threshold(None, 4, ctypes.c_float(0.5), None, None) == N.PSCA_EINVAL


def test_params_struct_layout_matches_header(tmp_path):
    """Field offsets and sizes of the ctypes mirrors against the C compiler's
    layout of include/psca.h."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in N.PscaParams._fields_]
    pfields = [f for f, _ in N.PscaProblem._fields_]
    bfields = [f for f, _ in N.PscaBackProblem._fields_]
    src = tmp_path / "layout.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "psca.h"', "int main(void) {",
             'printf("%zu %zu %zu\\n", sizeof(psca_params), sizeof(psca_problem), sizeof(psca_back_problem));']
    lines += [f'printf("%zu\\n", offsetof(psca_params, {f}));' for f in fields]
    lines += [f'printf("%zu\\n", offsetof(psca_problem, {f}));' for f in pfields]
    lines += [f'printf("%zu\\n", offsetof(psca_back_problem, {f}));' for f in bfields]
    lines += ["return 0; }"]
    src.write_text("\n".join(lines))
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(N.PscaParams)
    assert vals[1] == ctypes.sizeof(N.PscaProblem)
    assert vals[2] == ctypes.sizeof(N.PscaBackProblem)
    o = 3
    assert vals[o:o + len(fields)] == [getattr(N.PscaParams, f).offset for f in fields]
    o += len(fields)
    assert vals[o:o + len(pfields)] == [getattr(N.PscaProblem, f).offset for f in pfields]
    o += len(pfields)
    assert vals[o:] == [getattr(N.PscaBackProblem, f).offset for f in bfields]


def test_missing_library_fails_loudly(tmp_path):
    N2 = N
    saved = N2._lib
    try:
        N2._lib = None
        with pytest.raises(ImportError):
            N2.load(str(tmp_path / "nope.so"))
    finally:
        N2._lib = saved


def test_binding_module_imports_without_a_gpu():
    from paper_2503_15259_amd import psca
    assert psca.VARIANTS["MAP-UR"] == N.MAP_UR
    p = psca.Params(variant=N.ML_UD, iters=3, M=8).to_c()
    assert p.iters == 3 and p.g is None
