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
    st = lib.raft_ctx_create(0, None, ctypes.byref(h))
    assert st == _lib.E_DEVICE and not h.value


def test_product_path_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_2312_01560_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, re.M), f
                assert "oracle/" not in txt, f


def test_nmi_from_counts_host_finish():
    """raft_nmi_from_counts (host code of the library) against the oracle's
    NMI, itself pinned to scikit-learn: random label pairs, identical and
    permuted labelings (1.0), both constant (1.0)."""
    import numpy as np
    from oracle import scores
    from paper_2312_01560_amd import _lib
    lib = _lib.load()

    def via_lib(a, b):
        ka, kb = int(a.max()) + 1, int(b.max()) + 1
        counts = np.zeros((ka, kb), dtype=np.int64)
        np.add.at(counts, (a, b), 1)
        out = ctypes.c_double()
        st = lib.raft_nmi_from_counts(counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ka,
                                      kb, ctypes.byref(out))
        assert st == 0
        return out.value

    rng = np.random.default_rng(4)
    for n, ka, kb in ((1000, 5, 7), (5000, 40, 3), (300, 1, 9)):
        a = rng.integers(0, ka, n)
        b = rng.integers(0, kb, n)
        assert abs(via_lib(a, b) - scores.nmi(a, b)) < 1e-12
    a = rng.integers(0, 9, 2000)
    assert abs(via_lib(a, a) - 1.0) < 1e-12
    assert abs(via_lib(a, (a * 5 + 3) % 9) - 1.0) < 1e-12
    z = np.zeros(50, dtype=np.int64)
    assert via_lib(z, z) == 1.0
    bad = np.zeros((2, 2), dtype=np.int64)
    out = ctypes.c_double()
    assert lib.raft_nmi_from_counts(bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2, 2,
                                    ctypes.byref(out)) == _lib.E_INVAL
