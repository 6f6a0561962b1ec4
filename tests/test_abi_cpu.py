"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and reports the missing device as an error
instead of aborting."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raftgp.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(raft_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    from paper_2312_01560_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2312_01560_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.raft_abi_version() == _lib.ABI_VERSION
    assert lib.raft_status_string(-4) == b"workspace too small"


def test_config_struct_layout():
    from paper_2312_01560_amd import _lib
    # 19 int32 fields (76 bytes), padding to 8, then the uint64 seed
    assert _lib.RaftConfig.seed.offset == 80
    assert ctypes.sizeof(_lib.RaftConfig) == 88
    assert ctypes.sizeof(_lib.RaftOutputs) == 10 * 8


def test_no_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2312_01560_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.raft_ctx_create(0, ctypes.byref(h))
    assert st == _lib.E_DEVICE and not h.value


def test_product_path_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_2312_01560_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, re.M), f
                assert "oracle/" not in txt, f
