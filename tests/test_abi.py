"""The C-ABI library loads and exports every function include/sgrt.h declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sgrt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sg_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("sg_ctx_create", "sg_scene_create", "sg_solve", "sg_export_csr", "sg_trace", "sg_server_create",
              "sg_submit", "sg_poll", "sg_wait"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2503_16037_amd import sgrt
    L = ctypes.CDLL(sgrt.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    hdr = open(os.path.join(ROOT, "include", "sgrt.h")).read()
    version = int(re.search(r"#define SG_ABI_VERSION (\d+)u", hdr).group(1))
    assert L.sg_abi_version() == version == sgrt.ABI_VERSION


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2503_16037_amd import sgrt
    monkeypatch.setattr(sgrt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sgrt, "_lib", None)
    import pytest
    with pytest.raises(RuntimeError):
        sgrt.lib()
