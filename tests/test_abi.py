"""The C-ABI library loads on a host without a GPU and exports every entry
point declared in include/nqs.h (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nqs.h")
LIB = os.path.join(ROOT, "paper_2507_19276_amd", "libnqs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nqs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("nqs_ctx_create", "nqs_instance_create", "nqs_ansatz_create", "nqs_ansatz_bind_params",
              "nqs_eloc", "nqs_logpsi", "nqs_logpsi_vjp", "nqs_connected", "nqs_rows"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnqs.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnqs.so not built")
def test_host_only_calls_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.nqs_version.restype = ctypes.c_char_p
    assert lib.nqs_version().startswith(b"nqs-eloc")
    lib.nqs_last_error.restype = ctypes.c_char_p
    assert lib.nqs_last_error() is not None
    lib.nqs_instance_n_conn.restype = ctypes.c_int64
    assert lib.nqs_instance_n_conn(None) == -1
