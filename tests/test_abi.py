"""The C-ABI library loads and exports every function include/hrrm.h declares
(no compute without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hrrm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\**\s+\**(hrrm_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hrrm_median2d", "hrrm_median3d", "hrrm_ctx_create", "hrrm_rank2d",
                 "hrrm_median2d_batched", "hrrm_server_submit", "hrrm_autotune"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1105_3829_amd as hrrm
    if not os.path.exists(hrrm.LIB_PATH):
        pytest.skip("libhrrm.so not built")
    L = ctypes.CDLL(hrrm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(hrrm.EXPORTED_SYMBOLS) >= set(declared_functions())


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1105_3829_amd as hrrm
    monkeypatch.setattr(hrrm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hrrm, "_lib", None)
    with pytest.raises(ImportError):
        hrrm.lib()


def test_null_context_is_rejected_without_touching_a_device():
    import paper_1105_3829_amd as hrrm
    if not os.path.exists(hrrm.LIB_PATH):
        pytest.skip("libhrrm.so not built")
    L = hrrm.lib()
    assert L.hrrm_median2d(None, None, None, 1, 4, 4, 4, 4, 1, 0, None) == hrrm.EINVAL
    assert b"context" in L.hrrm_last_error()
    assert L.hrrm_ctx_create(0, None) == hrrm.EINVAL
    assert L.hrrm_ctx_destroy(None) == hrrm.OK
