"""The C ABI: the built library loads and exports every entry point that
include/rc.h declares, the header compiles as plain C, and the Python binding
covers the whole ABI.  No device calls (runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rc.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rc_[a-z_0-9]+)\s*\(", src)))


def test_header_compiles_as_c(tmp_path):
    c = tmp_path / "t.c"
    c.write_text('#include "rc.h"\nint main(void){ rc_sensor_desc d; rc_outputs o; (void)d; (void)o; return 0; }\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.dirname(HEADER),
                           "-c", str(c), "-o", str(tmp_path / "t.o")])


def test_binding_covers_abi():
    from paper_2503_01471_amd import rc
    assert sorted(rc.ABI) == declared()


def test_library_exports_every_symbol():
    from paper_2503_01471_amd import rc
    if not os.path.exists(rc.LIB_PATH):
        pytest.fail("librc.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(rc.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    # a call that touches no device
    L.rc_status_string.restype = ctypes.c_char_p
    assert L.rc_status_string(0) == b"ok"
    assert L.rc_status_string(-2) == b"out of memory"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2503_01471_amd import rc
    monkeypatch.setattr(rc, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(rc, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        rc.lib()
