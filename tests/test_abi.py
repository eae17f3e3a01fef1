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
    assert lib.psca_detect(None, None, None, 4, 4, ctypes.byref(prm), None, None, None) == N.PSCA_EINVAL
    assert lib.psca_detect_y(None, None, None, 4, 4, ctypes.byref(prm), None, None, None) == N.PSCA_EINVAL
    assert lib.psca_iterate(None, None, None, 4, 4, ctypes.byref(prm), ctypes.c_float(0.5), None, None,
                            None, None, None, None, None) == N.PSCA_EINVAL
    assert lib.psca_threshold(None, 4, ctypes.c_float(0.5), None, None) == N.PSCA_EINVAL


def test_params_struct_layout_matches_header():
    # int32 variant, int32 iters, float rho0, float rho_decay, ptr rho, float sigma2,
    # int32 M, ptr g, ptr p, 5 floats -> 4+4+4+4+8+4+4+8+8+20 = 68, padded to 72
    assert ctypes.sizeof(N.PscaParams) == 72
    assert N.PscaParams.rho.offset == 16 and N.PscaParams.g.offset == 32


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
