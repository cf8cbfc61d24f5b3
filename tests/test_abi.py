"""The C-ABI library loads and exports every symbol the header declares (CPU only:
no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2503_08854_amd", "libdtrack.so")


def declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(dt_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_entry_points():
    names = declared()
    for n in ("dt_ctx_create", "dt_patch_create", "dt_stack", "dt_topk", "dt_debug_samples"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdtrack.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dt_[a-z0-9_]+)$", out, flags=re.M))
    assert declared() <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdtrack.so not built")
def test_version_and_error_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.dt_version.restype = ctypes.c_char_p
    lib.dt_last_error.restype = ctypes.c_char_p
    assert b"gfx950" in lib.dt_version()
    assert lib.dt_last_error() == b""


def test_binding_names_match_header():
    import paper_2503_08854_amd.binding as b
    src = open(b.__file__).read()
    used = set(re.findall(r'"(dt_[a-z0-9_]+)"', src))
    assert used == declared()
