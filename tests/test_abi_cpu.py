"""The C ABI library builds, loads and exports what include/bz.h declares;
argument validation that happens before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def bz():
    import paper_1301_4195_amd as bz

    if not os.path.exists(bz.LIB_PATH):
        from paper_1301_4195_amd import build

        build.build()
    return bz


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("bz_op_create", "bz_op_destroy", "collision_eval", "conserve", "transport_step", "bz_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(bz):
    lib = ctypes.CDLL(bz.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) <= set(bz.EXPORTS) | {"bz_op_n"}


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1301_4195_amd as bzmod

    monkeypatch.setattr(bzmod, "_lib", None)
    monkeypatch.setattr(bzmod, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(bzmod.BzLibraryMissing):
        bzmod.load()


def test_validation_before_device_work(bz):
    lib = bz.load()
    h = ctypes.c_void_p()
    assert lib.bz_op_create(7, 6.0, 1.0, bz.BZ_F64, None, ctypes.byref(h)) == bz.BZ_EINVAL
    assert "N must be" in bz.bz_last_error()
    assert lib.bz_op_create(16, -1.0, 1.0, bz.BZ_F64, None, ctypes.byref(h)) == bz.BZ_EINVAL
    assert lib.bz_op_create(16, 6.0, -3.0, bz.BZ_F64, None, ctypes.byref(h)) == bz.BZ_EUNSUPPORTED
    assert lib.bz_op_create(16, 6.0, 1.0, 7, None, ctypes.byref(h)) == bz.BZ_EINVAL
    assert lib.bz_op_create(16, 6.0, 1.0, bz.BZ_F64, None, None) == bz.BZ_EINVAL
    assert lib.collision_eval(None, 1, None, None, bz.BZ_F64, None) == bz.BZ_EINVAL
    assert lib.conserve(None, 1, None, bz.BZ_F64, None, None, None) == bz.BZ_EINVAL
    assert lib.transport_step(None, 1, None, None, 0.1, None, None, None) == bz.BZ_EINVAL
    assert lib.bz_axpy(-1, 1.0, None, None, None) == bz.BZ_EINVAL
    assert lib.bz_axpy(0, 1.0, None, None, None) == bz.BZ_OK
    assert lib.bz_set_memory_cap(-5) == bz.BZ_EINVAL
    assert lib.bz_weights_gather(None, 1, None, None, None, None) == bz.BZ_EINVAL
    assert lib.bz_op_destroy(None) == bz.BZ_OK


def test_nonfinite_flag_constant_matches_header(bz):
    """The binding's copy of the non-finite moment flag is the header's."""
    import re

    text = open(os.path.join(ROOT, "include", "bz.h")).read()
    m = re.search(r"#define BZ_MOMENTS_NONFINITE_BITS (0x[0-9A-Fa-f]+)ull", text)
    assert m and int(m.group(1), 16) == bz.BZ_MOMENTS_NONFINITE_BITS
    flag = np.array([bz.BZ_MOMENTS_NONFINITE_BITS], dtype=np.uint64).view(np.float64)[0]
    assert np.isnan(flag)  # a quiet NaN: any test for a non-finite value finds it

